"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, its structs have the header's layout, and argument
validation rejects bad input before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2509_21754_amd import fitrig as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fitrig.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fitrig_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = F.load()
    names = header_functions()
    assert "fitrig_detect" in names and "fitrig_create" in names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", F.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}\b", out), n
    assert set(F.EXPORTS) == set(names)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "probe.c"
    exe = tmp_path / "probe"
    classes = {"fitrig_config": F.fitrig_config, "fitrig_candidate": F.fitrig_candidate,
               "fitrig_stats": F.fitrig_stats, "fitrig_server_config": F.fitrig_server_config,
               "fitrig_result": F.fitrig_result}
    fields = {k: [f for f, _ in c._fields_] for k, c in classes.items()}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fitrig.h"', "int main(void){"]
    for s, fs in fields.items():
        lines.append(f'printf("{s} size %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for s, cls in classes.items():
        assert got[(s, "size")] == ctypes.sizeof(cls), s
        for f, _ in cls._fields_:
            assert got[(s, f)] == getattr(cls, f).offset, (s, f)


def test_status_strings_and_version():
    assert F.fitrig_abi_version() == F.ABI_VERSION
    assert F.fitrig_status_string(F.OK) == "ok"
    for code in (F.E_INVAL, F.E_NOMEM, F.E_HIP, F.E_TRUNC, F.E_BUSY, F.E_NOTREADY, F.E_SCRATCH):
        assert F.fitrig_status_string(code) not in ("ok", "unknown status")
    assert F.fitrig_status_string(-99) == "unknown status"


def test_defaults():
    c = F.fitrig_config_default()
    assert (c.abi_version, c.mode, c.window, c.tile, c.branches, c.sigma_est, c.harm, c.r_signed,
            c.map_kind, c.C) == (F.ABI_VERSION, F.SLIDING, 7, 32, F.IMAGE | F.FREQ, F.MEAN_STD, 0, 0, F.MAP_QTILDE, 1e-6)


@pytest.mark.parametrize("bad", [
    dict(abi_version=F.ABI_VERSION + 1), dict(abi_version=1), dict(mode=2), dict(window=4), dict(window=0), dict(window=19), dict(tile=0),
    dict(branches=0), dict(branches=8), dict(branches=4, mode=1), dict(sigma_est=2), dict(harm=1), dict(harm=-1), dict(r_signed=2),
    dict(map_kind=3), dict(profile=2), dict(C=0.0), dict(C=-1.0), dict(C=float("nan")), dict(max_pixels=-1),
])
def test_create_rejects_bad_config(bad):
    rc, h = F.fitrig_create(F.fitrig_config_default(**bad))
    assert rc == F.E_INVAL and h is None


def test_detect_rejects_null_context():
    n = ctypes.c_int64(5)
    rc = F.fitrig_detect(None, ctypes.c_void_p(1), F.F32, 4, 8, 8, 6.0, None, 0, ctypes.byref(n), None, None, None,
                         None, None)
    assert rc == F.E_INVAL
    assert F.fitrig_destroy(None) == F.E_INVAL


def test_server_rejects_bad_config_on_cpu():
    for bad in (dict(n_slots=0), dict(max_fields=0), dict(cand_cap=-1), dict(mem_budget=-5), dict(window=2),
                dict(freq_window=-1), dict(freq_window=2049)):
        rc, h = F.fitrig_server_create(F.fitrig_server_config_default(**bad))
        assert rc == F.E_INVAL and h is None
    t = ctypes.c_int64()
    assert F.fitrig_submit(None, 0, ctypes.c_void_p(1), F.F32, 3, 4, 4, 6.0, 1, ctypes.byref(t)) == F.E_INVAL
    assert F.fitrig_poll(None, 1, 0, ctypes.byref(F.fitrig_result())) == F.E_INVAL
    assert F.fitrig_release(None, 1) == F.E_INVAL
    assert F.fitrig_server_destroy(None) == F.E_INVAL
    c = F.fitrig_server_config_default()
    assert (c.n_slots, c.max_fields, c.mem_budget, c.cand_cap, c.freq_window, c.base.window) == (4, 64, 0, 65536, 0, 7)


def test_interp_peaks_rejects_bad_arguments_on_cpu():
    import numpy as np

    py = np.array([1], np.int32)
    px = np.array([5], np.int32)
    out = np.zeros(3)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    dummy = ctypes.c_void_p(1)   # never dereferenced: arguments are checked first
    call = lambda *a: F.fitrig_interp_peaks(*a)    # noqa: E731
    assert call(dummy, 4, 4, p(py), p(px), 1, F.INTERP_SPLINE, 16, p(out), None) == F.E_INVAL   # x outside
    assert call(dummy, 4, 8, p(py), p(px), -1, F.INTERP_SPLINE, 16, p(out), None) == F.E_INVAL
    assert call(dummy, 4, 8, p(py), p(px), 1, 4, 16, p(out), None) == F.E_INVAL
    assert call(dummy, 4, 8, p(py), p(px), 1, F.INTERP_SPLINE, 0, p(out), None) == F.E_INVAL
    assert call(dummy, 4, 8, p(py), p(px), 1, F.INTERP_SPLINE, 65, p(out), None) == F.E_INVAL
    assert call(None, 4, 8, p(py), p(px), 1, F.INTERP_SPLINE, 16, p(out), None) == F.E_INVAL
    assert call(dummy, 0, 8, p(py), p(px), 1, F.INTERP_SPLINE, 16, p(out), None) == F.E_INVAL
    assert call(dummy, 4, 8, None, None, 0, F.INTERP_SPLINE, 16, None, None) == F.OK   # nothing to do


def test_noalloc_scratch_limit_matches_header():
    txt = open(HEADER).read()
    m = re.search(r"#define FITRIG_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == F.NOALLOC_SCRATCH_BYTES
    m = re.search(r"#define FITRIG_E_SCRATCH \((-\d+)\)", txt)
    assert m and int(m.group(1)) == F.E_SCRATCH
