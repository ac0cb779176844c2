"""Stacks in host memory streamed to the device in chunks of frames
(fitrig_detect_host, through the C ABI): every result equals the same stack
run from device memory, bit for bit, for chunk sizes from one frame to the
whole stack, pinned and pageable memory, FP32 / FP16, the median/MAD spread,
tile mode, and candidate truncation across chunks."""
import numpy as np
import pytest

from parity import structured_stack

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "f16": torch.float16}


def _stack(seed, n, H, W):
    X = structured_stack(seed, n, H, W)
    for k in range(1, n, 3):                   # periodic source for the frequency branch
        X[k, 40:47, 90:97] += 20.0
    return X


def _device_run(X, dt, tau, cand_cap, **cfg):
    from paper_2509_21754_amd import Context

    t = torch.from_numpy(X).to(DT[dt]).cuda()
    tile = cfg.get("tile", 32)
    eta = torch.full((-(-X.shape[1] // tile), -(-X.shape[2] // tile)), float("nan"), device="cuda")
    torch.cuda.synchronize()
    with Context(**cfg) as ctx:
        c, st, rc = ctx.detect(t, tau, cand_cap=cand_cap, eta_map=eta, as_dicts=False)
    return c, st, rc, eta.cpu().numpy()


def _host_run(X, dt, tau, chunk, pinned, cand_cap, **cfg):
    from paper_2509_21754_amd import Context

    h = torch.from_numpy(X).to(DT[dt])
    if pinned:
        h = h.pin_memory()
    tile = cfg.get("tile", 32)
    eta = torch.full((-(-X.shape[1] // tile), -(-X.shape[2] // tile)), float("nan"), device="cuda")
    torch.cuda.synchronize()
    with Context(**cfg) as ctx:
        c, st, rc = ctx.detect_host(h, tau, chunk, cand_cap=cand_cap, eta_map=eta, as_dicts=False)
    return c, st, rc, eta.cpu().numpy()


def _same(a, b):
    ca, sa, ra, ea = a
    cb, sb, rb, eb = b
    assert ra == rb
    assert ca.tobytes() == cb.tobytes()
    for k in ("M", "n_triples", "mu", "sigma", "flags", "eta_mu", "eta_sigma", "ran", "eta_flags", "n_image_cand",
              "n_freq_cand", "n_cand", "status"):
        assert sa[k] == sb[k], k
    assert ea.tobytes() == eb.tobytes()


@pytest.mark.parametrize("chunk", [1, 2, 3, 5, 14])
@pytest.mark.parametrize("pinned", [True, False])
def test_host_stream_equals_device(chunk, pinned):
    X = _stack(61, 14, 150, 300)
    cfg = dict(window=7, tile=16)
    ref = _device_run(X, "f32", 4.5, 1 << 14, **cfg)
    assert len(ref[0]) > 0 and ref[1]["n_freq_cand"] > 0
    _same(_host_run(X, "f32", 4.5, chunk, pinned, 1 << 14, **cfg), ref)


@pytest.mark.parametrize("cfg", [dict(window=9, sigma_est=1, tile=32), dict(mode=1, tile=8),
                                 dict(window=5, branches=1)])
def test_host_stream_other_forms(cfg):
    X = _stack(62, 11, 100, 260)
    for dt in ("f32", "f16"):
        ref = _device_run(X, dt, 4.5, 1 << 14, **cfg)
        _same(_host_run(X, dt, 4.5, 4, True, 1 << 14, **cfg), ref)


def test_host_stream_truncation_and_limits():
    from paper_2509_21754_amd import Context, FitrigError

    X = _stack(63, 12, 120, 300)
    ref = _device_run(X, "f32", 3.0, 1 << 14, window=7, tile=16)
    n_all = ref[1]["n_cand"]
    assert n_all > 6
    cap = n_all // 2
    got = _host_run(X, "f32", 3.0, 2, True, cap, window=7, tile=16)
    assert got[2] == -4 and got[1]["n_cand"] == n_all
    assert got[0].tobytes() == ref[0][:cap].tobytes()
    with Context(window=7, branches=4) as ctx:
        with pytest.raises(FitrigError):
            ctx.detect_host(torch.from_numpy(X), 3.0, 4)
