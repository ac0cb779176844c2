"""Builds the gfx950 HIP library ``libfitrig.so`` in place (hipcc).

The translation units compile in parallel: the runtime (which includes the
type-independent kernels), the serving loop, sub-cell localisation, and the
kernels templated on the storage type once per type.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfitrig.so")
ARCH = os.environ.get("FITRIG_OFFLOAD_ARCH", "gfx950")

# Packed FP32 ops are disabled for every HIP translation unit.
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-Wno-unused-result",
]

# (source, extra flags and defines, object name)
UNITS = [
    # the per-pixel transform's matrix products keep their loop-carried
    # accumulators in VGPRs (the default AGPR form copied all of them out and
    # back on every step of the series)
    ("fitrig_api.hip", ["-mllvm", "-amdgpu-mfma-vgpr-form"], "fitrig_api.o"),
    ("fitrig_server.hip", [], "fitrig_server.o"),
    ("fitrig_interp.hip", [], "fitrig_interp.o"),
    ("fitrig_accum.hip", [], "fitrig_accum.o"),
    ("fitrig_prefix.hip", [], "fitrig_prefix.o"),
    ("fitrig_launch.hip", ["-DFITRIG_STORAGE=0"], "fitrig_launch_f32.o"),
    ("fitrig_launch.hip", ["-DFITRIG_STORAGE=1"], "fitrig_launch_f16.o"),
    ("fitrig_launch.hip", ["-DFITRIG_STORAGE=2"], "fitrig_launch_bf16.o"),
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra: list[str] | None = None, jobs: int | None = None) -> str:
    cc = hipcc()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="fitrig_build_") as tmpd:
        def compile_unit(u):
            src, defs, obj = u
            cmd = [cc, *HIPCC_FLAGS, *(extra or []), *defs, *inc, "-c", os.path.join(CSRC, src),
                   "-o", os.path.join(tmpd, obj)]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src} {defs}:\n{msg}")
            if verbose and msg.strip():
                print(msg, flush=True)
            return os.path.join(tmpd, obj)

        n = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=n) as ex:
            objs = list(ex.map(compile_unit, UNITS))
        tmp = LIB + ".tmp"
        # roctx: named ranges of the launch phases for rocprofv3 --marker-trace
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread",
               "-lrocprofiler-sdk-roctx"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
