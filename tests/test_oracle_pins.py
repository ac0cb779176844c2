"""Pins of the FP64 oracle against values fixed by the paper and by
mathematics, not by the oracle itself: hand-worked examples (tests/golden),
library special cases (scipy.ndimage, numpy.fft, numpy.median), closed forms.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import ref


def test_worked_example_1_tile_mode(golden):
    g = golden("worked_example_1.json")
    X = np.array(g["frames"], float)
    d, r = ref.pixel_terms(X, 0)
    np.testing.assert_array_equal(d, g["delta"])
    np.testing.assert_allclose(r, g["r"], rtol=0, atol=0)
    q = ref.index_maps(X, mode=ref.TILES, tile=g["tile"])
    assert q.shape == (1, 1, 1)
    assert q[0, 0, 0] == pytest.approx(g["q"], rel=1e-15)
    # Eq. (6) sum form: sum(D) max(D) sum(r) / (N_T^2)^2
    assert g["sum_delta"] * g["max_delta"] * g["sum_r"] / 16.0 == pytest.approx(q[0, 0, 0], rel=1e-15)
    M = ref.normaliser(X, g["C"])
    assert M == g["M"]
    assert 1 - q[0, 0, 0] / M**2 == pytest.approx(g["tlisi"], rel=1e-15)


def test_worked_example_1_signed_reading(golden):
    g = golden("worked_example_1.json")["signed_variant"]
    X = np.array(g["frames"], float)
    d, r_abs = ref.pixel_terms(X, 0, r_signed=False)
    _, r_sig = ref.pixel_terms(X, 0, r_signed=True)
    np.testing.assert_array_equal(d, g["delta"])
    np.testing.assert_array_equal(r_abs, g["r_abs"])
    np.testing.assert_array_equal(r_sig, g["r_signed"])
    qa = ref.index_maps(X, mode=ref.TILES, tile=2)[0, 0, 0]
    qs = ref.index_maps(X, mode=ref.TILES, tile=2, r_signed=True)[0, 0, 0]
    assert qa == pytest.approx(g["q_abs"], rel=1e-15)
    assert qs == pytest.approx(g["q_signed"], rel=1e-15)
    M = ref.normaliser(X)
    assert 1 - qs / M**2 == pytest.approx(g["tlisi_signed"], rel=1e-15)


def test_worked_example_2_per_pixel_zscore(golden):
    g = golden("worked_example_2.json")
    X = np.array(g["frames"], float)
    q = ref.index_maps(X, mode=ref.SLIDING, window=g["window"])
    np.testing.assert_allclose(q[0], g["q"], rtol=1e-15)
    np.testing.assert_allclose(1 - q[0] / 25.0, g["tlisi"], rtol=1e-15)
    mu, sig = ref.spread(q[0])
    assert mu == pytest.approx(g["mu"], rel=1e-15)
    assert sig == pytest.approx(g["sigma"], rel=1e-14)
    np.testing.assert_allclose((q[0] - mu) / sig, g["z"], atol=1e-7)
    comps = ref.components(q[0], mu, sig, g["tau"])
    assert [(c["peak_y"], c["peak_x"]) for c in comps] == [tuple(p) for p in g["selected"]]
    out = ref.detect(X, tau=g["tau"], window=1, branches=ref.IMAGE)
    assert len(out["cands"]) == 1 and out["cands"][0]["label"] == 1


def test_worked_example_3_clipped_window(golden):
    g = golden("worked_example_3.json")
    X = np.array(g["frames"], float)
    d, r = ref.pixel_terms(X, 0)
    np.testing.assert_array_equal(d, g["delta"])
    np.testing.assert_array_equal(r, g["r"])
    q = ref.index_maps(X, mode=ref.SLIDING, window=g["window"])
    np.testing.assert_allclose(q[0], g["q"], rtol=1e-15)
    assert ref.normaliser(X) == g["M"]


def test_zero_reference_uses_C(golden):
    g = golden("zero_reference.json")
    X = np.array(g["frames"], float)
    d, r = ref.pixel_terms(X, 0, C=g["C"])
    np.testing.assert_allclose(d, g["delta"], rtol=1e-12)
    np.testing.assert_allclose(r, g["r"], rtol=1e-12)
    q = ref.index_maps(X, window=1, C=g["C"])
    np.testing.assert_allclose(q[0], g["q"], rtol=1e-12)


def test_ccl_example(golden):
    g = golden("ccl_example.json")
    z = np.array(g["z"], float)
    comps = ref.components(z, 0.0, 1.0, g["tau"])
    assert len(comps) == len(g["components"])
    for c, e in zip(comps, g["components"]):
        for k, v in e.items():
            assert c[k] == pytest.approx(v, rel=1e-14), (k, c, e)


def test_spectrum_closed_form(golden):
    g = golden("spectrum_example.json")
    n = g["nprime"]
    s = np.arange(n)
    v = g["offset"] + sum(a * np.cos(2 * np.pi * k * s / n) for k, a in g["terms"])
    cube = v.reshape(n, 1, 1)
    assert ref.eta(cube, 0)[0, 0] == pytest.approx(g["eta_max"], rel=1e-12)
    assert ref.eta(cube, 2)[0, 0] == pytest.approx(g["eta_hsum2"], rel=1e-12)
    # constant series -> eta = 0
    assert ref.eta(np.full((n, 1, 1), 7.0), 0)[0, 0] == pytest.approx(0.0, abs=1e-12)


def test_spread_examples(golden):
    g = golden("spread_example.json")
    for key in ("odd", "even"):
        med, sig = ref.spread(np.array(g[key]["values"], float), ref.MEDIAN_MAD)
        assert med == g[key]["median"]
        assert sig == pytest.approx(g["scale"] * g[key]["mad"], rel=1e-15)
    # the scale is 1 / Phi^-1(3/4)
    from scipy.stats import norm

    assert g["scale"] == pytest.approx(1.0 / norm.ppf(0.75), rel=1e-12)


# ---- library special cases ------------------------------------------------

def _rand_stack(rng, n, H, W, zeros=False):
    X = rng.normal(size=(n, H, W))
    X[:, rng.integers(0, H, 3), rng.integers(0, W, 3)] += 20.0
    if zeros:
        X[rng.random((n, H, W)) < 0.05] = 0.0
    return X


@pytest.mark.parametrize("shape,w", [((5, 13, 17), 3), ((4, 9, 20), 7), ((3, 8, 5), 9), ((6, 31, 11), 5)])
def test_sliding_windows_match_scipy(shape, w):
    """Window sums / max over the clipped window equal scipy's zero-padded
    box filters (Delta, r >= 0 so padding with 0 is neutral), and the count
    equals the box filter of ones."""
    rng = np.random.default_rng(sum(shape) + w)
    X = _rand_stack(rng, *shape, zeros=True)
    q = ref.index_maps(X, window=w)
    for s in range(shape[0] - 2):
        d, r = ref.pixel_terms(X, s)
        ones = np.ones_like(d)
        cnt = ndimage.correlate(ones, np.ones((w, w)), mode="constant", cval=0.0)
        sd = ndimage.correlate(d, np.ones((w, w)), mode="constant", cval=0.0)
        sr = ndimage.correlate(r, np.ones((w, w)), mode="constant", cval=0.0)
        md = ndimage.maximum_filter(d, size=w, mode="constant", cval=0.0)
        np.testing.assert_allclose(q[s], (sd / cnt) * md * (sr / cnt), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("shape,w", [((5, 13, 17), 3), ((4, 9, 20), 9)])
def test_index_cells_match_scipy(shape, w):
    """The per-cell sampler (used for sampled parity at full size, also on
    crops) equals the same scipy box filters at every cell, edges included."""
    rng = np.random.default_rng(7 * sum(shape) + w)
    X = _rand_stack(rng, *shape, zeros=True)
    n, H, W = shape
    cells = np.array([(s, y, x) for s in range(n - 2) for y in range(H) for x in range(W)])
    got = ref.index_cells(X, cells, window=w).reshape(n - 2, H, W)
    for s in range(n - 2):
        d, r = ref.pixel_terms(X, s)
        cnt = ndimage.correlate(np.ones_like(d), np.ones((w, w)), mode="constant", cval=0.0)
        sd = ndimage.correlate(d, np.ones((w, w)), mode="constant", cval=0.0)
        sr = ndimage.correlate(r, np.ones((w, w)), mode="constant", cval=0.0)
        md = ndimage.maximum_filter(d, size=w, mode="constant", cval=0.0)
        np.testing.assert_allclose(got[s], (sd / cnt) * md * (sr / cnt), rtol=1e-12, atol=1e-15)
    # a crop holding a cell's clipped window gives the same value
    for s, y, x in cells[::37]:
        ya, yb, xa, xb = max(0, y - w // 2), min(H, y + w // 2 + 1), max(0, x - w // 2), min(W, x + w // 2 + 1)
        c = ref.index_cells(np.ascontiguousarray(X[s:s + 3, ya:yb, xa:xb]), [[0, y - ya, x - xa]], window=w)[0]
        assert c == got[s, y, x]


@pytest.mark.parametrize("shape,t", [((4, 12, 10), 4), ((3, 9, 13), 4), ((5, 7, 7), 1), ((3, 33, 70), 32)])
def test_tile_mode_matches_block_reduction(shape, t):
    rng = np.random.default_rng(shape[1] * 7 + t)
    X = _rand_stack(rng, *shape)
    q = ref.index_maps(X, mode=ref.TILES, tile=t)
    H, W = shape[1:]
    Ty, Tx = -(-H // t), -(-W // t)
    assert q.shape == (shape[0] - 2, Ty, Tx)
    for s in range(shape[0] - 2):
        d, r = ref.pixel_terms(X, s)
        for ty in range(Ty):
            for tx in range(Tx):
                bd = d[ty * t:(ty + 1) * t, tx * t:(tx + 1) * t]
                br = r[ty * t:(ty + 1) * t, tx * t:(tx + 1) * t]
                assert q[s, ty, tx] == pytest.approx(bd.mean() * bd.max() * br.mean(), rel=1e-12)


def test_eta_matches_numpy_rfft():
    rng = np.random.default_rng(3)
    for npr in (4, 5, 14, 30, 31, 62, 65, 126, 127, 130):
        cube = rng.normal(size=(npr, 3, 4)) + 5.0
        e = ref.eta(cube, 0)
        v = cube - cube.mean(0, keepdims=True)
        A = np.abs(np.fft.rfft(v, axis=0))[1:npr // 2 + 1]
        np.testing.assert_allclose(e, A.max(0), rtol=1e-10)
        # harmonic sum of 3 terms from the same magnitudes
        K = npr // 2
        hs = np.stack([sum(A[j * k - 1] for j in range(1, 4) if j * k <= K) for k in range(1, K + 1)])
        np.testing.assert_allclose(ref.eta(cube, 3), hs.max(0), rtol=1e-10)


def test_spread_matches_numpy():
    rng = np.random.default_rng(4)
    for n in (1, 2, 7, 100, 1001):
        v = rng.gamma(2.0, size=n)
        mu, sig = ref.spread(v, ref.MEAN_STD)
        assert mu == pytest.approx(v.mean(), rel=1e-13)
        assert sig == pytest.approx(v.std(ddof=0), rel=1e-12, abs=1e-15)
        med, s2 = ref.spread(v, ref.MEDIAN_MAD)
        assert med == np.median(v)
        assert s2 == pytest.approx(1.482602218505602 * np.median(np.abs(v - np.median(v))), rel=1e-15)


def test_components_match_scipy_label():
    rng = np.random.default_rng(5)
    for trial in range(20):
        H, W = rng.integers(1, 40, 2)
        z = rng.normal(size=(H, W)) * 2
        tau = 1.0
        comps, mask = ref.components(z, 0.0, 1.0, tau, with_mask=True)
        np.testing.assert_array_equal(mask, z > tau)
        lab, nl = ndimage.label(z > tau, structure=np.ones((3, 3)))
        assert nl == len(comps)
        seen = {}
        for c in comps:
            l = lab.flat[c["label"]]
            assert l > 0 and l not in seen
            seen[l] = c
            ys, xs = np.nonzero(lab == l)
            lin = ys * W + xs
            assert c["label"] == lin.min()
            assert c["n_pix"] == len(ys)
            w = z[ys, xs]
            best = np.lexsort((lin, -w))[0]
            assert (c["peak_y"], c["peak_x"]) == (ys[best], xs[best])
            assert c["cy"] == pytest.approx((w * ys).sum() / w.sum(), rel=1e-12)
            assert c["cx"] == pytest.approx((w * xs).sum() / w.sum(), rel=1e-12, abs=1e-12)
            assert (c["y0"], c["x0"], c["y1"], c["x1"]) == (ys.min(), xs.min(), ys.max(), xs.max())
        # canonical order: increasing label
        assert [c["label"] for c in comps] == sorted(c["label"] for c in comps)


# ---- closed forms ------------------------------------------------------------

@pytest.mark.parametrize("tau,q", [(3.0, 1.3498980316301e-3), (4.0, 3.1671241833120e-5)])
def test_threshold_stage_gaussian_tail(tau, q):
    """Fed an N(0,1) map, the N-sigma selection keeps a fraction within a
    binomial interval of the Gaussian tail Q(tau)."""
    rng = np.random.default_rng(int(tau * 10))
    N = 2_000_000
    v = rng.normal(size=(1000, N // 1000))
    mu, sig = ref.spread(v)
    _, mask = ref.components(v, mu, sig, tau, with_mask=True)
    frac = mask.mean()
    assert q == pytest.approx(0.5 * math.erfc(tau / math.sqrt(2)), rel=1e-9)
    tol = 5 * math.sqrt(q * (1 - q) / N) + 2e-6 * q * 0
    assert abs(frac - q) < tol, (frac, q, tol)


def test_mad_sigma_consistent_on_gaussian():
    rng = np.random.default_rng(11)
    N = 400_000
    v = rng.normal(size=N)
    _, sig = ref.spread(v, ref.MEDIAN_MAD)
    assert abs(sig - 1.0) < 5 * 1.17 / math.sqrt(N)


# ---- sub-cell peak localisation (oracle/interp.py) --------------------------

def test_interp_spline_and_makima_match_scipy():
    from scipy.interpolate import Akima1DInterpolator, CubicSpline

    from oracle import interp as I

    rng = np.random.default_rng(11)
    x = np.arange(5.0)
    ts = np.linspace(0.0, 4.0, 57)
    for _ in range(20):
        f = rng.normal(size=5) * rng.uniform(0.1, 10.0)
        got_s = np.array([I.interp1(f, t, I.SPLINE) for t in ts])
        got_m = np.array([I.interp1(f, t, I.MAKIMA) for t in ts])
        assert np.allclose(got_s, CubicSpline(x, f)(ts), rtol=1e-12, atol=1e-12)
        assert np.allclose(got_m, Akima1DInterpolator(x, f, method="makima")(ts), rtol=1e-12, atol=1e-12)


def test_interp_methods_pass_through_nodes_and_reproduce_polynomials():
    from oracle import interp as I

    rng = np.random.default_rng(12)
    f = rng.normal(size=5)
    for meth in (I.BILINEAR, I.BICUBIC, I.SPLINE, I.MAKIMA):
        for k in range(5):
            assert I.interp1(f, float(k), meth) == pytest.approx(f[k], abs=1e-14)
    lin = [0.5 + 1.25 * k for k in range(5)]
    quad = [-(k - 2.3) ** 2 + 5.0 for k in range(5)]
    cub = [0.1 * k ** 3 - k ** 2 + 2.0 for k in range(5)]
    for t in np.linspace(1.0, 3.0, 17):
        for meth in (I.BILINEAR, I.BICUBIC, I.SPLINE, I.MAKIMA):
            assert I.interp1(lin, t, meth) == pytest.approx(0.5 + 1.25 * t, abs=1e-12)
        # Keys' kernel (a = -1/2) is exact for quadratics away from the ends;
        # the not-a-knot spline for cubics
        assert I.interp1(quad, t, I.BICUBIC) == pytest.approx(-(t - 2.3) ** 2 + 5.0, abs=1e-12)
        assert I.interp1(cub, t, I.SPLINE) == pytest.approx(0.1 * t ** 3 - t ** 2 + 2.0, abs=1e-12)
    # Keys' weights are a partition of unity
    for t in np.linspace(0.0, 1.0, 11):
        assert sum(I.keys_weight(t - k) for k in range(-1, 3)) == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("y0,x0", [(10.25, 7.5), (9.8125, 8.0625), (10.0, 8.0)])
def test_interp_peak_of_a_quadratic_surface_is_exact(y0, x0):
    """A separable quadratic peak sampled on the cells: bicubic and spline
    reproduce it, so the grid maximum is the true peak (on the 1/16 grid)."""
    from oracle import interp as I

    yy, xx = np.mgrid[0:20, 0:16].astype(np.float64)
    m = 100.0 - 1.5 * (yy - y0) ** 2 - 0.75 * (xx - x0) ** 2
    py, px = int(round(y0)), int(round(x0))
    for meth in (I.BICUBIC, I.SPLINE):
        y, x, v = I.interp_peak(m, py, px, meth, sub=16)
        assert (y, x) == (y0, x0)
        assert v == pytest.approx(100.0, abs=1e-9)
    # bilinear surfaces peak at a node
    y, x, _ = I.interp_peak(m, py, px, I.BILINEAR, sub=16)
    assert y == int(y) and x == int(x)


def test_interp_peak_ties_and_edges():
    from oracle import interp as I

    m = np.full((6, 7), 3.0)
    # a flat bilinear surface: every grid value ties, the first (a, b) wins
    assert I.interp_peak(m, 2, 3, I.BILINEAR, sub=4)[:2] == (1.0, 2.0)
    # at a corner the neighbourhood repeats the edge cells: a peak cell with
    # higher neighbours on the inside moves inward
    m = np.zeros((6, 7))
    m[0, 0], m[0, 1], m[1, 0], m[1, 1] = 5.0, 4.0, 4.0, 3.0
    y, x, _ = I.interp_peak(m, 0, 0, I.SPLINE, sub=8)
    assert -1.0 <= y <= 1.0 and -1.0 <= x <= 1.0
    F = I.neighbourhood(m, 0, 0)
    assert F[0, 0] == F[2, 2] == 5.0 and F[4, 4] == 0.0


def test_per_pixel_frequency_branch_equals_tile_one_with_window_one():
    """With a 1 x 1 window the sliding maps are the 1 x 1 tile cube, so the
    per-pixel spectrum, its spread and its components are the tile branch's."""
    rng = np.random.default_rng(21)
    X = rng.normal(size=(14, 20, 23)) + 5.0
    X[::3, 8:11, 4:7] += 6.0
    for sigma_est in (ref.MEAN_STD, ref.MEDIAN_MAD):
        out = ref.detect(X, tau=3.0, window=1, tile=1, branches=ref.FREQ | ref.FREQ_PIXEL, sigma_est=sigma_est)
        assert np.allclose(out["eta_px"], out["eta"], rtol=1e-12, atol=0.0)
        assert out["eta_px_mu"] == pytest.approx(out["eta_mu"], rel=1e-12)
        assert out["eta_px_sigma"] == pytest.approx(out["eta_sigma"], rel=1e-12)
        a = [{k: v for k, v in c.items() if k != "branch"} for c in out["cands"] if c["branch"] == ref.FREQ]
        b = [{k: v for k, v in c.items() if k != "branch"} for c in out["cands"] if c["branch"] == ref.FREQ_PIXEL]
        assert a and len(a) == len(b)
        for u, v in zip(a, b):
            assert u.keys() == v.keys()
            for k in u:
                assert u[k] == pytest.approx(v[k], rel=1e-9, abs=1e-12), k


def test_per_pixel_frequency_branch_finds_a_periodic_pixel_source():
    rng = np.random.default_rng(22)
    X = rng.normal(size=(34, 40, 48)) + 10.0
    X[1::4, 20:23, 30:33] += 8.0    # period 4 snapshots
    out = ref.detect(X, tau=6.0, window=3, branches=ref.FREQ_PIXEL)
    c = [c for c in out["cands"] if c["branch"] == ref.FREQ_PIXEL]
    assert c and all(c_["triple"] == -1 for c_ in c)
    best = max(c, key=lambda c_: c_["peak_z"])
    assert 18 <= best["peak_y"] <= 24 and 28 <= best["peak_x"] <= 34
    # fewer than four triples: the branch does not run (as the tile branch)
    assert ref.detect(X[:5], tau=6.0, window=3, branches=ref.FREQ_PIXEL)["eta_px"] is None


@pytest.mark.parametrize("n", [6, 67, 128])
def test_per_pixel_spectrum_matches_numpy_rfft_any_length(n):
    """The per-pixel eta is the one-sided magnitude maximum of the DFT of each
    cell's mean-removed q series (Eq. (10) applied per cell), for every series
    length, including lengths past 64 and odd ones: pinned to numpy's FFT of
    the oracle's own q maps."""
    rng = np.random.default_rng(n)
    X = rng.normal(size=(n, 9, 13)) + 4.0
    X[2::5, 3:6, 4:8] += 5.0
    out = ref.detect(X, tau=3.0, window=3, branches=ref.IMAGE | ref.FREQ_PIXEL)
    q = out["q"]
    v = q - q.mean(0, keepdims=True)
    A = np.abs(np.fft.rfft(v, axis=0))[1:(n - 2) // 2 + 1]
    np.testing.assert_allclose(out["eta_px"], A.max(0), rtol=1e-10)
    mu, sig = A.max(0).mean(), A.max(0).std()
    assert out["eta_px_mu"] == pytest.approx(mu, rel=1e-10)
    assert out["eta_px_sigma"] == pytest.approx(sig, rel=1e-10)
