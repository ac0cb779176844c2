"""GPU parity on the full 4096 x 4096 x 64 FP32 workload (window 7,
thresholds 5, 6, 7) against the whole FP64 oracle, and on seeded 2048 x 2048
crops of the 50000 x 50000 x 16 FP16 workload (window 9, tau 6): crop-interior
q against the oracle on the same decoded FP16 values, and every candidate of
the full-image run inside a crop's interior against the oracle's component
built with the full-image mean and std (the oracle cannot see the global
statistics of a 50000^2 image)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import ref
from parity import Z_BAND, check_candidates, check_eta, check_maps, check_stats

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1200)]


def _cands_at(out, tau):
    """The oracle's candidate list at another threshold, from the same maps and statistics."""
    o = dict(out)
    o["cands"] = []
    for s in range(out["q"].shape[0]):
        if out["flags"][s]:
            continue
        for c in ref.components(out["q"][s], out["mu"][s], out["sigma"][s], tau):
            c.update(branch=ref.IMAGE, triple=s)
            o["cands"].append(c)
    if out.get("eta") is not None and out["eta_sigma"] > 0:
        for c in ref.components(out["eta"], out["eta_mu"], out["eta_sigma"], tau):
            c.update(branch=ref.FREQ, triple=-1)
            o["cands"].append(c)
    return o


def test_c1_full_against_oracle():
    import synth
    from paper_2509_21754_amd import Context

    spec = synth.WORKLOADS["c1"]
    assert (spec.n, spec.H, spec.W, spec.window) == (64, 4096, 4096, 7)
    print("[c1] generating 64 x 4096 x 4096", flush=True)
    stack = synth.make_stack(spec, device="cuda")
    torch.cuda.synchronize()
    Ty = -(-spec.H // 32)
    qmap = torch.empty((spec.n - 2, spec.H, spec.W), device="cuda")
    eta = torch.empty((Ty, Ty), device="cuda")
    runs = {}
    with Context(window=spec.window, max_pixels=spec.H * spec.W, max_snap=spec.n) as ctx:
        for tau in spec.taus:
            runs[tau] = ctx.detect(stack, tau, index_map=qmap, eta_map=eta)
    torch.cuda.synchronize()
    X = stack.cpu().numpy()
    del stack
    print("[c1] oracle", flush=True)
    out = ref.detect(X.astype(np.float64), tau=spec.taus[0], window=spec.window)
    del X
    check_maps(qmap.cpu().numpy(), out["q"])
    check_eta(eta.cpu().numpy(), out["eta"])
    for tau in spec.taus:
        cands, stats, rc = runs[tau]
        assert rc == 0
        check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"], out["flags"])
        assert stats["eta_mu"] == pytest.approx(out["eta_mu"], rel=1e-6)
        assert stats["eta_sigma"] == pytest.approx(out["eta_sigma"], rel=1e-6)
        n = check_candidates(cands, _cands_at(out, tau), tau)
        print(f"[c1] tau {tau}: {len(cands)} candidates, {n} compared", flush=True)
        assert n > 0


def _component_at(q2, mu, sg, tau, py, px):
    comps, mask = ref.components(q2, mu, sg, tau, with_mask=True)
    if not mask[py, px]:
        return None
    lab, _ = ndimage.label(mask, structure=np.ones((3, 3)))
    first = int(np.flatnonzero(lab.ravel() == lab[py, px])[0])
    return next(d for d in comps if d["label"] == first)


def test_c3_crops():
    import synth
    from paper_2509_21754_amd import Context

    spec = synth.WORKLOADS["c3"]
    assert (spec.n, spec.H, spec.W, spec.window, spec.dtype) == (16, 50000, 50000, 9, "f16")
    print("[c3] generating 16 x 50000 x 50000 fp16", flush=True)
    stack = synth.make_stack(spec, device="cuda")
    torch.cuda.synchronize()
    tau = spec.taus[0]
    h = spec.window // 2
    CROP = 2048
    lo, hi = h, CROP - h
    with Context(window=spec.window, max_pixels=spec.H * spec.W, max_snap=spec.n) as ctx:
        cands, stats, rc = ctx.detect(stack, tau, cand_cap=1 << 21, as_dicts=False)
    assert rc == 0
    img = cands[cands["branch"] == ref.IMAGE]
    checked = 0
    for i in range(3):
        rng = np.random.default_rng(3000 + i)
        oy = 16 * int(rng.integers(0, (spec.H - CROP) // 16 + 1))
        ox = 16 * int(rng.integers(0, (spec.W - CROP) // 16 + 1))
        sub = stack[:, oy:oy + CROP, ox:ox + CROP].contiguous()
        qg = torch.empty((spec.n - 2, CROP, CROP), device="cuda")
        with Context(window=spec.window) as ctx:
            ctx.detect(sub, tau, index_map=qg, as_dicts=False)
        qg = qg.cpu().numpy()[:, lo:hi, lo:hi]
        qd = ref.index_maps(sub.float().cpu().numpy(), window=spec.window)[:, lo:hi, lo:hi]
        check_maps(qg, qd, what=f"crop {i}")
        inside = img[(img["y0"] >= oy + lo + 1) & (img["y1"] < oy + hi - 1) &
                     (img["x0"] >= ox + lo + 1) & (img["x1"] < ox + hi - 1)]
        for c in inside:
            s = int(c["triple"])
            mu, sg = stats["mu"][s], stats["sigma"][s]
            y0, y1 = int(c["y0"]) - oy - lo - 1, int(c["y1"]) - oy - lo + 2
            x0, x1 = int(c["x0"]) - ox - lo - 1, int(c["x1"]) - ox - lo + 2
            if np.any(np.abs((qd[s][y0:y1, x0:x1] - mu) / sg - tau) <= Z_BAND):
                continue
            py, px = int(c["peak_y"]) - oy - lo - y0, int(c["peak_x"]) - ox - lo - x0
            d = _component_at(qd[s][y0:y1, x0:x1], mu, sg, tau, py, px)
            assert d is not None, (i, s, c["label"])
            assert (d["n_pix"], d["y0"] + y0, d["x0"] + x0, d["y1"] + y0, d["x1"] + x0) == (
                int(c["n_pix"]), int(c["y0"]) - oy - lo, int(c["x0"]) - ox - lo, int(c["y1"]) - oy - lo,
                int(c["x1"]) - ox - lo), (i, s, c["label"])
            checked += 1
        print(f"[c3] crop {i} at ({oy}, {ox}): {len(inside)} candidates inside", flush=True)
    assert checked > 0
