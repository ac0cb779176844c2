"""The allocation-free entry (fitrig_detect_noalloc, scratch in the library's
static device array) against fitrig_detect on the same inputs, through the C
ABI: identical candidates, statistics and maps, on two calls in a row (the
second with a smaller stack), and the size limit as an error."""
import ctypes

import numpy as np
import pytest

from parity import structured_stack

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _call(fn, ctx, t, tau, cand_cap, with_maps, tile=32):
    from paper_2509_21754_amd import fitrig as F

    n, H, W = t.shape
    np_ = n - 2
    cand = (F.fitrig_candidate * cand_cap)()
    ncand = ctypes.c_int64(-1)
    mu = (ctypes.c_double * np_)()
    sg = (ctypes.c_double * np_)()
    fl = (ctypes.c_uint32 * np_)()
    st = F.fitrig_stats()
    st.mu = ctypes.cast(mu, ctypes.POINTER(ctypes.c_double))
    st.sigma = ctypes.cast(sg, ctypes.POINTER(ctypes.c_double))
    st.flags = ctypes.cast(fl, ctypes.POINTER(ctypes.c_uint32))
    qmap = torch.full((np_, H, W), float("nan"), device="cuda") if with_maps else None
    eta = torch.full((-(-H // tile), -(-W // tile)), float("nan"), device="cuda") if with_maps else None
    ptr = lambda m: ctypes.c_void_p(m.data_ptr()) if m is not None else None  # noqa: E731
    torch.cuda.synchronize()
    rc = fn(ctx, ctypes.c_void_p(t.data_ptr()), F._dtype_code(t), n, H, W, float(tau), cand, cand_cap,
            ctypes.byref(ncand), ptr(qmap), ptr(eta), None, ctypes.byref(st), None)
    torch.cuda.synchronize()
    k = max(0, min(ncand.value, cand_cap))
    recs = bytes(memoryview(cand).cast("B")[: k * ctypes.sizeof(F.fitrig_candidate)])
    scal = (st.M, st.n_triples, st.status, st.eta_mu, st.eta_sigma, st.n_image_cand, st.n_freq_cand, st.ran,
            st.eta_flags)
    maps = (qmap.cpu().numpy().tobytes(), eta.cpu().numpy().tobytes()) if with_maps else None
    return rc, ncand.value, recs, list(mu), list(sg), list(fl), scal, maps


def _stacks():
    a = structured_stack(41, 12, 300, 700)
    for k in range(2, 12, 3):
        a[k, 100:107, 200:207] += 25.0
    b = structured_stack(42, 7, 90, 260)
    b[3, 40:45, 100:105] += 30.0
    return a, b


@pytest.mark.parametrize("cfg", [dict(window=7), dict(window=9, sigma_est=1), dict(mode=1, tile=8)])
def test_noalloc_equals_detect_two_calls(cfg):
    from paper_2509_21754_amd import Context
    from paper_2509_21754_amd import fitrig as F

    a, b = _stacks()
    with Context(**cfg) as ref_ctx, Context(**cfg) as na_ctx:
        for X, with_maps in ((a, True), (b, False)):
            t = torch.from_numpy(X).cuda()
            if cfg.get("mode", 0) == 1 and with_maps:
                with_maps = False  # tile-mode maps have the tile shape; compared through the candidates
            r = _call(F.fitrig_detect, ref_ctx.handle, t, 5.0, 4096, with_maps)
            g = _call(F.fitrig_detect_noalloc, na_ctx.handle, t, 5.0, 4096, with_maps)
            assert r[0] == 0 and g[0] == 0, (r[0], g[0])
            assert r[1] > 0
            assert g[1:] == r[1:]
        # the context's own path still works after the allocation-free calls
        t = torch.from_numpy(a).cuda()
        assert _call(F.fitrig_detect, na_ctx.handle, t, 5.0, 4096, True)[1:] == \
            _call(F.fitrig_detect, ref_ctx.handle, t, 5.0, 4096, True)[1:]


def test_noalloc_rejects_a_call_beyond_the_array():
    from paper_2509_21754_amd import Context
    from paper_2509_21754_amd import fitrig as F

    # median/MAD without an index map needs an [n-2][H][W] float map in scratch:
    # 18 x 2048 x 2048 -> 16 * 4 Mi * 4 B = 256 MiB, beyond the array with the rest
    X = torch.randn((18, 2048, 2048), device="cuda")
    with Context(window=7, sigma_est=1) as ctx:
        rc = _call(F.fitrig_detect_noalloc, ctx.handle, X, 5.0, 16, False)[0]
        assert rc == F.E_SCRATCH
        assert F.fitrig_status_string(rc) != "unknown status"
        # and a small call afterwards runs
        t = torch.from_numpy(_stacks()[1]).cuda()
        assert _call(F.fitrig_detect_noalloc, ctx.handle, t, 5.0, 16, False)[0] in (0, F.E_TRUNC)
