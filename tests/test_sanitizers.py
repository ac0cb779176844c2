"""AddressSanitizer and UndefinedBehaviorSanitizer builds on the CPU: the FP64
oracle's C library run through its pins, and the host runtime's argument
checks, sizing passes and result unpacking fuzzed over shapes and
configurations (host code only; no GPU is used)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = tmp_path / "libfitrig_ref_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", *SAN,
                           os.path.join(ROOT, "oracle", "fitrig_ref.c"), "-o", str(lib), "-lm"])
    env = dict(os.environ, FITRIG_REF_LIB=str(lib), LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run(["python3", os.path.join(ROOT, "tests", "sanitize", "oracle_driver.py")], env=env,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_host_runtime_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "host_sizing"
    cmd = [hipcc, "-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops"]
    for f in SAN:
        cmd += ["-Xarch_host", f]
    cmd += ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2509_21754_amd", "csrc"),
            os.path.join(ROOT, "tests", "sanitize", "host_sizing.cpp"), "-o", str(exe), "-lrocprofiler-sdk-roctx"]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "failures" in r.stdout and " 0 failures" in r.stdout
