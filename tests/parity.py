"""Helpers for GPU-vs-oracle parity (imported by the GPU tests).

Tolerances (from the workload statement, made concrete):
  index maps     |q_gpu - q_ref| <= 1e-5 |q_ref| + 1e-7 mean|q_ref| (per triple); q_ref == 0 -> exactly 0
  mu, sigma      <= 1e-6 relative
  candidates     identical cell sets except cells with |z_ref - tau| <= 1e-4; compared per
                 component: label, n_pix, bbox exact; peak exact unless the oracle's top two
                 values in the component are within 1e-5 relative; centroid within 1e-4 cell
  eta            |eta_gpu - eta_ref| <= 1e-5 eta_ref (+1e-12 absolute)
"""
from __future__ import annotations

import numpy as np

from oracle import ref

MAP_RTOL = 1e-5
MAP_ATOL_REL_MEAN = 1e-7
STAT_RTOL = 1e-6
Z_BAND = 1e-4
CENTROID_TOL = 1e-4
ETA_RTOL = 1e-5


def check_maps(q_gpu: np.ndarray, q_ref: np.ndarray, what: str = "q"):
    q_gpu = np.asarray(q_gpu, np.float64)
    assert q_gpu.shape == q_ref.shape, (q_gpu.shape, q_ref.shape)
    for s in range(q_ref.shape[0]):
        r = q_ref[s]
        g = q_gpu[s]
        tol = MAP_RTOL * np.abs(r) + MAP_ATOL_REL_MEAN * np.abs(r).mean()
        bad = np.abs(g - r) > tol
        assert not bad.any(), (
            f"{what}[{s}]: {bad.sum()} cells outside tolerance; worst rel "
            f"{(np.abs(g - r) / np.maximum(np.abs(r), 1e-300)).max():.3e}")
        assert np.all(g[r == 0.0] == 0.0), f"{what}[{s}]: exact zeros not preserved"


def check_stats(mu_g, sig_g, mu_r, sig_r, flags_r=None):
    for s in range(len(mu_r)):
        if flags_r is not None and flags_r[s]:
            continue
        assert abs(mu_g[s] - mu_r[s]) <= STAT_RTOL * abs(mu_r[s]) + 1e-300, (s, mu_g[s], mu_r[s])
        assert abs(sig_g[s] - sig_r[s]) <= STAT_RTOL * abs(sig_r[s]) + 1e-300, (s, sig_g[s], sig_r[s])


def _near_border(c, border_mask):
    H, W = border_mask.shape
    y0, y1 = max(c["y0"] - 1, 0), min(c["y1"] + 2, H)
    x0, x1 = max(c["x0"] - 1, 0), min(c["x1"] + 2, W)
    return border_mask[y0:y1, x0:x1].any()


def check_components(gpu: list, refc: list, values_ref: np.ndarray, mu: float, sigma: float, tau: float,
                     where: str = ""):
    """Compare the components of one set (triple or eta grid)."""
    z = (values_ref - mu) / sigma
    border = np.abs(z - tau) <= Z_BAND
    labels = None
    g_by = {c["label"]: c for c in gpu}
    r_by = {c["label"]: c for c in refc}
    if not border.any():
        assert [c["label"] for c in gpu] == [c["label"] for c in refc], (where, len(gpu), len(refc))
    n_checked = 0
    for lab, rc in r_by.items():
        if _near_border(rc, border):
            continue
        assert lab in g_by, (where, "missing component", rc)
        gc = g_by[lab]
        for k in ("n_pix", "y0", "x0", "y1", "x1"):
            assert gc[k] == rc[k], (where, k, gc, rc)
        # cells of this component (other components may share its box),
        # looked at inside the box only
        if labels is None:
            from scipy import ndimage

            labels, _ = ndimage.label(z > tau, structure=np.ones((3, 3)))
        y0, y1, x0, x1 = rc["y0"], rc["y1"] + 1, rc["x0"], rc["x1"] + 1
        own = labels[y0:y1, x0:x1] == labels[rc["peak_y"], rc["peak_x"]]
        vals = values_ref[y0:y1, x0:x1]
        top = vals[own].max()
        near = (vals >= top * (1 - 1e-5)) if top > 0 else (vals >= top * (1 + 1e-5))
        allowed = {(int(a) + y0, int(b) + x0) for a, b in np.argwhere(own & near)}
        assert (gc["peak_y"], gc["peak_x"]) in allowed, (where, "peak", gc, rc)
        if len(allowed) == 1:
            assert (gc["peak_y"], gc["peak_x"]) == (rc["peak_y"], rc["peak_x"])
        assert abs(gc["cy"] - rc["cy"]) <= CENTROID_TOL and abs(gc["cx"] - rc["cx"]) <= CENTROID_TOL, (where, gc, rc)
        assert abs(gc["peak_z"] - rc["peak_z"]) <= 1e-4 * max(1.0, abs(rc["peak_z"])), (where, gc, rc)
        n_checked += 1
    for lab, gc in g_by.items():
        if lab not in r_by:
            assert _near_border(gc, border), (where, "extra component", gc)
    return n_checked


def check_candidates(cands: list, out: dict, tau: float, *, image_values=None):
    """Compare a whole GPU candidate list with the oracle's detect() output."""
    keys = [(c["branch"], c["triple"], c["label"]) for c in cands]
    assert keys == sorted(keys, key=lambda k: (k[0], k[1] if k[0] == ref.IMAGE else 0, k[2])), "order"
    img_vals = out["q"] if image_values is None else image_values
    nchk = 0
    if img_vals is not None:
        for s in range(img_vals.shape[0]):
            if out["flags"][s]:
                assert not [c for c in cands if c["branch"] == ref.IMAGE and c["triple"] == s]
                continue
            g = [c for c in cands if c["branch"] == ref.IMAGE and c["triple"] == s]
            r = [c for c in out["cands"] if c["branch"] == ref.IMAGE and c["triple"] == s]
            nchk += check_components(g, r, img_vals[s], out["mu"][s], out["sigma"][s], tau, where=f"triple {s}")
    if out.get("eta") is not None and out["eta_sigma"] and out["eta_sigma"] > 0:
        g = [c for c in cands if c["branch"] == ref.FREQ]
        r = [c for c in out["cands"] if c["branch"] == ref.FREQ]
        nchk += check_components(g, r, out["eta"], out["eta_mu"], out["eta_sigma"], tau, where="freq")
    if out.get("eta_px") is not None and out["eta_px_sigma"] and out["eta_px_sigma"] > 0:
        g = [c for c in cands if c["branch"] == ref.FREQ_PIXEL]
        r = [c for c in out["cands"] if c["branch"] == ref.FREQ_PIXEL]
        nchk += check_components(g, r, out["eta_px"], out["eta_px_mu"], out["eta_px_sigma"], tau,
                                 where="freq per pixel")
    else:
        assert not [c for c in cands if c["branch"] == ref.FREQ_PIXEL]
    return nchk


def check_eta(eta_gpu, eta_ref):
    g = np.asarray(eta_gpu, np.float64)
    bad = np.abs(g - eta_ref) > ETA_RTOL * np.abs(eta_ref) + 1e-12
    assert not bad.any(), f"eta: {bad.sum()} tiles outside tolerance, worst {np.abs(g - eta_ref).max():.3e}"


def structured_stack(seed: int, n: int, H: int, W: int, dtype=np.float32, pulse_amp: float = 12.0,
                     steady_amp: float = 150.0, zeros: bool = False):
    """Noise + a few steady Gaussian sources + single-frame pulses (inputs
    with real candidates in several triples)."""
    import synth

    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, H, W))
    core = synth.gaussian_core(7)
    def stamp(img, y, x, a):
        ya, yb = max(0, y - 3), min(H, y + 4)
        xa, xb = max(0, x - 3), min(W, x + 4)
        img[ya:yb, xa:xb] += a * core[ya - (y - 3):yb - (y - 3), xa - (x - 3):xb - (x - 3)]
    S = np.zeros((H, W))
    for _ in range(max(1, H * W // 4000)):
        stamp(S, int(rng.integers(0, H)), int(rng.integers(0, W)), steady_amp * rng.uniform(0.2, 1))
    X += S
    for k in range(n):
        for _ in range(max(1, H * W // 6000)):
            if rng.random() < 0.6:
                stamp(X[k], int(rng.integers(0, H)), int(rng.integers(0, W)), pulse_amp * rng.uniform(0.5, 1.5))
    if zeros:
        X[rng.random(X.shape) < 0.02] = 0.0
    return X.astype(dtype)
