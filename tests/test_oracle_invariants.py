"""Invariants of the method checked on the FP64 oracle (exact in FP64), and
the recovery fixtures the design claims (Sec. 2.2.1: the index is high when
neither or both difference images hold the pulse; Sec. 2.2.3: the clamped
ratio suppresses bright steady structure)."""
import numpy as np
import pytest

from oracle import ref
import synth


def noise_stack(seed, n=8, H=40, W=48):
    return np.random.default_rng(seed).normal(size=(n, H, W))


def test_I1_identical_frames_give_nothing():
    rng = np.random.default_rng(1)
    f = rng.normal(size=(30, 34)) * 5 + 100.0
    X = np.stack([f] * 6)
    out = ref.detect(X, window=5, tau=3.0, branches=ref.IMAGE | ref.FREQ)
    assert np.all(out["q"] == 0.0)
    assert out["cands"] == []
    assert all(fl == ref.FLAG_SIGMA_ZERO for fl in out["flags"])
    assert np.all(out["cube"] == 0.0) and np.all(out["eta"] == 0.0)


def test_I2_steady_image_leaves_delta_unchanged():
    X = noise_stack(2)
    S = np.zeros(X.shape[1:])
    S[10:20, 5:9] = 200.0
    S[30, 40] = -50.0
    for s in range(X.shape[0] - 2):
        d0, r0 = ref.pixel_terms(X, s)
        d1, r1 = ref.pixel_terms(X + S, s)
        np.testing.assert_allclose(d1, d0, rtol=0, atol=1e-12)
        ref_ = X[s + 1] + S
        np.testing.assert_allclose(r1, np.minimum(d0 / np.abs(ref_), 1.0), rtol=1e-12, atol=1e-14)
        assert np.all(r1[S == 200.0] < 0.1)


@pytest.mark.parametrize("k", [-3, 4])
def test_I3_power_of_two_scaling(k):
    X = noise_stack(3)
    a = 2.0**k
    o1 = ref.detect(X, window=5, tau=2.5)
    o2 = ref.detect(X * a, window=5, tau=2.5, C=1e-6 * a)
    np.testing.assert_array_equal(o2["q"], o1["q"] * a * a)
    assert [(c["triple"], c["label"], c["n_pix"]) for c in o1["cands"]] == \
           [(c["triple"], c["label"], c["n_pix"]) for c in o2["cands"]]
    np.testing.assert_allclose(np.array(o2["sigma"]), np.array(o1["sigma"]) * a * a, rtol=1e-13)


def test_I4_time_reversal():
    X = noise_stack(4, n=10)
    q = ref.index_maps(X, window=3)
    qr = ref.index_maps(X[::-1].copy(), window=3)
    np.testing.assert_allclose(qr, q[::-1], rtol=1e-14)
    c = ref.index_maps(X, mode=ref.TILES, tile=8)
    cr = ref.index_maps(X[::-1].copy(), mode=ref.TILES, tile=8)
    np.testing.assert_allclose(ref.eta(cr), ref.eta(c), rtol=1e-10)


def test_I5_transpose_and_flip():
    X = noise_stack(5, H=23, W=31)
    q = ref.index_maps(X, window=5)
    qt = ref.index_maps(np.ascontiguousarray(X.transpose(0, 2, 1)), window=5)
    np.testing.assert_allclose(qt, q.transpose(0, 2, 1), rtol=1e-14)
    qf = ref.index_maps(np.ascontiguousarray(X[:, ::-1, :]), window=5)
    np.testing.assert_allclose(qf, q[:, ::-1, :], rtol=1e-14)


@pytest.mark.parametrize("w", [1, 3, 5, 7])
def test_I6_sliding_sampled_at_tile_centres_equals_tile_mode(w):
    X = noise_stack(6, H=4 * w + 2, W=3 * w + 1)
    q = ref.index_maps(X, window=w)
    t = ref.index_maps(X, mode=ref.TILES, tile=w)
    h = w // 2
    H, W = X.shape[1:]
    for ty in range(H // w):
        for tx in range(W // w):
            np.testing.assert_allclose(q[:, ty * w + h, tx * w + h], t[:, ty, tx], rtol=1e-14)


def _pulse_stack(seed, p=5, amp=10.0, n=9, H=48, W=48, steady=None):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, H, W))
    core = synth.gaussian_core(9)
    py, px = 24, 24
    X[p, py - 4:py + 5, px - 4:px + 5] += amp * core
    if steady is not None:
        sy, sx, sa = steady
        S = np.zeros((H, W))
        S[sy - 4:sy + 5, sx - 4:sx + 5] += sa * core
        X += S
    return X, (py, px)


def test_I7_single_frame_pulse_trigger_pattern():
    """A pulse confined to frame p changes D(p-1) and D(p): triples p-2 and p
    hold it in one difference image only (low index, high z); triple p-1
    holds it in both (the change cancels to the noise level)."""
    p = 5
    for seed in range(4):
        X, (py, px) = _pulse_stack(seed, p=p)
        out = ref.detect(X, window=7, tau=6.0, branches=ref.IMAGE)
        q = out["q"]
        z = [(q[s] - out["mu"][s]) / out["sigma"][s] for s in range(q.shape[0])]
        assert z[p - 2][py, px] > 6 and z[p][py, px] > 6
        assert z[p - 1][py, px] < 6
        hit = {c["triple"] for c in out["cands"]
               if abs(c["peak_y"] - py) <= 4 and abs(c["peak_x"] - px) <= 4}
        assert {p - 2, p} <= hit and (p - 1) not in hit


def test_recovery_pulsar_20x_fainter_than_steady_neighbour():
    """Peak 10 sigma pulse 8 px from a steady source of 200 (20x brighter),
    7x7 window, tau = 6: found in both trigger triples for every seed."""
    p = 4
    for seed in range(6):
        X, (py, px) = _pulse_stack(100 + seed, p=p, steady=(24, 32, 200.0))
        out = ref.detect(X, window=7, tau=6.0, branches=ref.IMAGE)
        hit = {c["triple"] for c in out["cands"]
               if abs(c["peak_y"] - py) <= 3 and abs(c["peak_x"] - px) <= 3}
        assert {p - 2, p} <= hit, (seed, hit)


def test_steady_source_gives_no_trigger():
    """Noise plus a bright steady source: nothing is selected on the source."""
    for seed in range(5):
        rng = np.random.default_rng(200 + seed)
        X = rng.normal(size=(10, 48, 48))
        X[:, 20:29, 20:29] += 500.0 * synth.gaussian_core(9)
        out = ref.detect(X, window=7, tau=6.0, branches=ref.IMAGE)
        near = [c for c in out["cands"] if 18 <= c["peak_y"] <= 30 and 18 <= c["peak_x"] <= 30]
        assert near == []


def test_frequency_branch_finds_periodic_tile():
    """A source pulsing every 4th frame in one tile gives the largest eta,
    selected by the z-score on eta (Eqs. (10)-(12))."""
    rng = np.random.default_rng(9)
    n, H, W, t = 34, 64, 96, 16
    X = rng.normal(size=(n, H, W))
    core = synth.gaussian_core(9)
    for k in range(2, n, 4):
        X[k, 36:45, 52:61] += 6.0 * core
    out = ref.detect(X, tile=t, window=7, tau=3.0, branches=ref.FREQ)
    e = out["eta"]
    ty, tx = np.unravel_index(np.argmax(e), e.shape)
    assert (ty, tx) == (40 // t, 56 // t)
    freq = [c for c in out["cands"] if c["branch"] == ref.FREQ]
    assert any(c["y0"] <= ty <= c["y1"] and c["x0"] <= tx <= c["x1"] for c in freq)


def test_workload_c0_runs_on_oracle():
    """The small workload end to end (shapes, ordering, flags)."""
    X = synth.make_stack(synth.WORKLOADS["c0"]).numpy()
    out = ref.detect(X, window=7, tau=6.0)
    assert out["q"].shape == (30, 256, 256)
    assert out["eta"].shape == (8, 8)
    keys = [(c["branch"], c["triple"], c["label"]) for c in out["cands"]]
    assert keys == sorted(keys, key=lambda k: (k[0], k[1], k[2]))
