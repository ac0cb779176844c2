"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle
on the same seeded inputs, at sizes that span several workgroup tiles and
ragged tails, plus edge cases and determinism."""
import numpy as np
import pytest

from oracle import ref
from parity import (check_candidates, check_eta, check_maps, check_stats, structured_stack)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def _ctx(**cfg):
    from paper_2509_21754_amd import Context

    return Context(**cfg)


def run_gpu(X, tau, dtype="f32", with_maps=True, cand_cap=1 << 16, eta_px=False, **cfg):
    """X: float32/float64 numpy stack -> (cands, stats, qmap, eta, stack used, status); with
    eta_px=True the per-pixel eta map is returned in stats["eta_px_map"]."""
    t = torch.from_numpy(np.ascontiguousarray(X)).to(DT[dtype]).cuda()
    n, H, W = t.shape
    mode = cfg.get("mode", 0)
    tile = cfg.get("tile", 32)
    if mode == 0:
        qshape = (n - 2, H, W)
    else:
        qshape = (n - 2, -(-H // tile), -(-W // tile))
    qmap = torch.full(qshape, float("nan"), device="cuda") if with_maps else None
    eta = torch.full((-(-H // tile), -(-W // tile)), float("nan"), device="cuda") if with_maps else None
    epx = torch.full((H, W), float("nan"), device="cuda") if eta_px else None
    with _ctx(**cfg) as ctx:
        cands, stats, rc = ctx.detect(t, tau, index_map=qmap, eta_map=eta, eta_px_map=epx, cand_cap=cand_cap)
    torch.cuda.synchronize()
    used = t.float().cpu().numpy()
    if eta_px:
        stats["eta_px_map"] = epx.cpu().numpy()
    return cands, stats, (qmap.cpu().numpy() if with_maps else None), (eta.cpu().numpy() if with_maps else None), used, rc


SMALL = [
    # (H, W, n, window, dtype, seed)
    (37, 530, 5, 7, "f32", 1),
    (70, 249, 6, 9, "f32", 2),
    (16, 16, 3, 1, "f32", 3),
    (5, 7, 4, 3, "f32", 4),
    (33, 300, 7, 5, "f16", 5),
    (48, 260, 8, 17, "bf16", 6),
    (90, 760, 4, 11, "f32", 7),
    (1, 600, 4, 7, "f32", 8),
    (600, 1, 4, 7, "f32", 9),
    (1, 1, 3, 1, "f32", 10),
    (129, 497, 6, 15, "f32", 11),
    (64, 512, 5, 3, "f32", 12),
]


@pytest.mark.parametrize("H,W,n,w,dt,seed", SMALL)
def test_sliding_parity_small(H, W, n, w, dt, seed):
    X = structured_stack(seed, n, H, W)
    tau = 3.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, dt, window=w, branches=1)
    assert rc == 0
    out = ref.detect(used, tau=tau, window=w, branches=ref.IMAGE)
    check_maps(q, out["q"])
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"], out["flags"])
    assert [int(f) for f in stats["flags"]] == out["flags"]
    check_candidates(cands, out, tau)
    assert stats["M"] == pytest.approx(ref.normaliser(used), rel=0, abs=0)


@pytest.mark.parametrize("zeros", [False, True])
def test_both_branches_parity(zeros):
    X = structured_stack(21, 14, 150, 700, zeros=zeros)
    for k in range(2, 14, 4):
        X[k, 60:67, 300:307] += 30.0
    tau = 4.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=7)
    assert rc == 0
    out = ref.detect(used, tau=tau, window=7)
    check_maps(q, out["q"])
    check_eta(eta, out["eta"])
    assert stats["eta_mu"] == pytest.approx(out["eta_mu"], rel=1e-6)
    assert stats["eta_sigma"] == pytest.approx(out["eta_sigma"], rel=1e-6)
    n = check_candidates(cands, out, tau)
    assert n > 0
    assert any(c["branch"] == ref.FREQ for c in cands)


def test_workload_c0():
    import synth

    spec = synth.WORKLOADS["c0"]
    X = synth.make_stack(spec).numpy()
    cands, stats, q, eta, used, rc = run_gpu(X, 6.0, window=7)
    out = ref.detect(used, tau=6.0, window=7)
    check_maps(q, out["q"])
    check_eta(eta, out["eta"])
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])
    check_candidates(cands, out, 6.0)


@pytest.mark.parametrize("tau", [5.0, 6.0, 7.0])
def test_workload_c1_crop(tau):
    import synth

    spec = synth.spec("c1", H=384, W=800, n=64)
    X = synth.make_stack(spec).numpy()
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=7)
    out = ref.detect(used, tau=tau, window=7)
    check_maps(q, out["q"])
    check_eta(eta, out["eta"])
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])
    check_candidates(cands, out, tau)


@pytest.mark.parametrize("tile,H,W,n", [(32, 100, 300, 8), (5, 37, 53, 6), (1, 9, 11, 4), (64, 70, 300, 6),
                                        (7, 64, 512, 5), (8, 203, 777, 7), (2, 70, 530, 5), (16, 260, 1030, 6),
                                        (4, 33, 257, 9)])
def test_tile_mode_parity(tile, H, W, n):
    X = structured_stack(30 + tile, n, H, W)
    tau = 2.5
    cands, stats, q, eta, used, rc = run_gpu(X, tau, mode=1, tile=tile)
    out = ref.detect(used, tau=tau, mode=ref.TILES, tile=tile)
    check_maps(q, out["q"])
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"], out["flags"])
    check_candidates(cands, out, tau)
    if out["eta"] is not None:
        check_eta(eta, out["eta"])


def test_median_mad_parity():
    X = structured_stack(41, 9, 80, 520)
    tau = 5.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=5, sigma_est=1)
    out = ref.detect(used, tau=tau, window=5, sigma_est=ref.MEDIAN_MAD)
    check_maps(q, out["q"])
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])
    check_candidates(cands, out, tau)


def test_median_mad_odd_count():
    """Odd cell count per triple: the middle order statistic is one value."""
    X = structured_stack(43, 7, 37, 53)
    tau = 3.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=3, sigma_est=1)
    out = ref.detect(used, tau=tau, window=3, sigma_est=ref.MEDIAN_MAD)
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])
    check_candidates(cands, out, tau)


def test_median_mad_ties():
    """A periodic stack gives q maps whose values repeat many times: the two
    middle order statistics (even count) and the MAD land inside runs of equal
    values."""
    rng = np.random.default_rng(44)
    n, H, W = 8, 64, 256
    tileval = rng.normal(size=(n, 8, 8)) * 2.0 + 5.0
    X = np.tile(tileval, (1, H // 8, W // 8)).astype(np.float32)
    tau = 2.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=1, sigma_est=1, branches=1)
    out = ref.detect(used, tau=tau, window=1, sigma_est=ref.MEDIAN_MAD, branches=ref.IMAGE)
    check_maps(q, out["q"])
    assert len(np.unique(q[0])) <= 64
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])
    check_candidates(cands, out, tau)


@pytest.mark.parametrize("W", [4096, 4097])
def test_median_mad_large_sets(W):
    """Sets of more than 8 * 2^20 cells take the sample-bracket-gather
    selection (even and odd counts)."""
    rng = np.random.default_rng(W)
    X = (rng.normal(size=(4, 4096, W)) + 3.0).astype(np.float32)
    tau = 10.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=3, sigma_est=1, branches=1, with_maps=False)
    out = ref.detect(used, tau=tau, window=3, sigma_est=ref.MEDIAN_MAD, branches=ref.IMAGE)
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])
    assert rc == 0
    check_candidates(cands, out, tau)


def test_median_mad_large_unaligned():
    """A set of more than 8 * 2^20 cells whose count is odd and not a
    multiple of 4: the bracket pass reads it one value at a time."""
    rng = np.random.default_rng(4099)
    X = (rng.normal(size=(3, 2049, 4097)) + 3.0).astype(np.float32)
    tau = 10.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=3, sigma_est=1, branches=1, with_maps=False)
    out = ref.detect(used, tau=tau, window=3, sigma_est=ref.MEDIAN_MAD, branches=ref.IMAGE, keep_maps=False)
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])


def test_median_mad_large_periodic():
    """A map periodic along rows at the sampling stride: the strided sample
    sees one phase only, the bracket misses and the full selection runs."""
    rng = np.random.default_rng(45)
    tileval = rng.normal(size=(4, 8, 8)) * 2.0 + 5.0
    X = np.tile(tileval, (1, 512, 512)).astype(np.float32)
    tau = 2.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=1, sigma_est=1, branches=1, with_maps=False)
    out = ref.detect(used, tau=tau, window=1, sigma_est=ref.MEDIAN_MAD, branches=ref.IMAGE, keep_maps=False)
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])


def test_median_mad_tiles_and_freq():
    X = structured_stack(42, 12, 96, 320)
    tau = 3.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, mode=1, tile=8, sigma_est=1)
    out = ref.detect(used, tau=tau, mode=ref.TILES, tile=8, sigma_est=ref.MEDIAN_MAD)
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])
    assert stats["eta_mu"] == pytest.approx(out["eta_mu"], rel=1e-6)
    assert stats["eta_sigma"] == pytest.approx(out["eta_sigma"], rel=1e-6)
    check_candidates(cands, out, tau)


@pytest.mark.parametrize("harm", [0, 3])
def test_freq_branch_only(harm):
    X = structured_stack(51, 34, 64, 300)
    for k in range(1, 34, 5):
        X[k, 20:27, 100:107] += 9.0
    tau = 3.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, branches=2, harm=harm, tile=16)
    out = ref.detect(used, tau=tau, branches=ref.FREQ, harm=harm, tile=16)
    check_eta(eta, out["eta"])
    check_candidates(cands, out, tau)
    assert all(c["branch"] == ref.FREQ and c["triple"] == -1 for c in cands)


@pytest.mark.parametrize("n,harm", [(200, 0), (200, 4), (303, 3)])
def test_freq_branch_long_series(n, harm):
    """Tile branch on series of n' >= 128 (a workgroup per tile): eta per tile
    against the oracle, candidates by component; H, W not multiples of the
    tile."""
    rng = np.random.default_rng(n + harm)
    X = structured_stack(70 + n, n, 45, 110)
    period = int(rng.integers(5, 12))
    for k in range(0, n, period):
        X[k, 10:15, 40:46] += 8.0
    tau = 3.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, branches=2, harm=harm, tile=16)
    assert rc == 0
    out = ref.detect(used, tau=tau, branches=ref.FREQ, harm=harm, tile=16)
    check_eta(eta, out["eta"])
    check_candidates(cands, out, tau)
    assert any(c["branch"] == ref.FREQ for c in cands)


@pytest.mark.parametrize("n,harm", [(6, 0), (34, 0), (34, 2), (35, 0), (66, 3), (67, 0)])
def test_freq_branch_register_series(n, harm):
    """Tile branch on series of n' <= 64 (each tile's series held in
    registers, in two sizes: up to 32 and up to 64 values, both ends of each
    and a harmonic sum): eta per tile against the oracle, candidates by
    component; H, W not multiples of the tile."""
    rng = np.random.default_rng(900 + n + harm)
    X = structured_stack(500 + n, n, 50, 90)
    period = int(rng.integers(3, 7))
    for k in range(0, n, period):
        X[k, 20:25, 30:36] += 8.0
    tau = 3.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, branches=2, harm=harm, tile=8)
    assert rc == 0
    out = ref.detect(used, tau=tau, branches=ref.FREQ, harm=harm, tile=8)
    check_eta(eta, out["eta"])
    check_candidates(cands, out, tau)


def test_r_signed_reading():
    X = structured_stack(61, 6, 40, 280)
    X -= 1.0
    tau = 3.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=5, r_signed=1, branches=1)
    out = ref.detect(used, tau=tau, window=5, r_signed=True, branches=ref.IMAGE)
    check_maps(q, out["q"])
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"])
    check_candidates(cands, out, tau)


def test_tlisi_map_kind():
    X = structured_stack(71, 5, 30, 270)
    t = torch.from_numpy(X).cuda()
    qmap = torch.empty((3, 30, 270), device="cuda")
    with _ctx(window=3, map_kind=1, branches=1) as ctx:
        cands, stats, rc = ctx.detect(t, 4.0, index_map=qmap)
    q = ref.index_maps(X, window=3)
    M = ref.normaliser(X)
    np.testing.assert_allclose(qmap.cpu().numpy(), 1 - q / M**2, rtol=0, atol=2e-7)


@pytest.mark.parametrize("w,dt", [(3, "f32"), (5, "f16"), (9, "f32"), (9, "bf16"), (13, "f32"), (17, "f32")])
def test_recompute_matches_stream_bitwise(w, dt):
    """The q of the selected segments, evaluated again for their cells, is the
    streaming pass's q bit for bit (one arithmetic, Eqs. (3)-(6)): every
    image candidate's peak q equals the q map at its peak cell. A low tau
    gives peaks at every row position of the 8-row blocks, in ragged bands
    and column groups."""
    X = structured_stack(300 + w, 7, 200, 700)
    cands, stats, q, eta, used, rc = run_gpu(X, 2.5, dtype=dt, window=w, branches=1)
    assert rc == 0
    img = [c for c in cands if c["branch"] == ref.IMAGE]
    assert len(img) > 50
    assert {c["peak_y"] % 8 for c in img} == set(range(8))
    for c in img:
        assert np.float32(c["peak_q"]) == q[c["triple"], c["peak_y"], c["peak_x"]], c


def test_components_across_slot_seams():
    """8-connected components whose cells cross the 64-cell slot seams and
    the column-group seams (window 3: groups of 254 cells), compared with
    the oracle's labelling: diagonal lines both ways, a run along a row,
    a U whose arms join below, and shapes meeting at one corner."""
    rng = np.random.default_rng(404)
    n, H, W = 6, 64, 700
    X = rng.normal(size=(n, H, W))
    img = np.zeros((H, W))
    for x0 in (60, 124, 250, 315):
        for t in range(12):
            img[4 + t, x0 + t] = 40.0           # down-right diagonal over the seam
            img[30 + t, x0 + 8 - t] = 40.0      # down-left diagonal over the seam
        img[20, x0 - 6:x0 + 10] = 40.0          # run along a row over the seam
        img[44:52, x0 - 2] = 40.0               # U: two arms ...
        img[44:52, x0 + 6] = 40.0
        img[52, x0 - 2:x0 + 7] = 40.0           # ... joined below
    img[57:60, 61:64] = 40.0                     # two squares meeting at a corner
    img[60:63, 64:67] = 40.0                     # on the seam at x = 64
    X[3] += img
    tau = 5.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, window=3, branches=1)
    assert rc == 0
    out = ref.detect(used, tau=tau, window=3, branches=ref.IMAGE)
    check_maps(q, out["q"])
    n_chk = check_candidates(cands, out, tau)
    assert n_chk >= 12


def test_determinism_bitwise():
    X = structured_stack(81, 10, 120, 600)
    r1 = run_gpu(X, 3.0, window=9)
    r2 = run_gpu(X, 3.0, window=9)
    assert r1[0] == r2[0]
    assert np.array_equal(r1[2], r2[2]) and np.array_equal(r1[3], r2[3], equal_nan=True)
    assert r1[1]["mu"] == r2[1]["mu"] and r1[1]["sigma"] == r2[1]["sigma"]


def test_identical_frames_give_nothing():
    f = np.random.default_rng(3).normal(size=(50, 300)).astype(np.float32) * 5 + 100
    X = np.stack([f] * 7)
    cands, stats, q, eta, used, rc = run_gpu(X, 3.0, window=5)
    assert cands == [] and rc == 0
    assert np.all(q == 0.0)
    assert all(fl & 1 for fl in stats["flags"])


def test_power_of_two_scaling_bitwise():
    X = structured_stack(91, 6, 64, 300).astype(np.float32)
    a = np.float32(4.0)
    r1 = run_gpu(X, 3.0, window=7, branches=1, C=1e-6)
    r2 = run_gpu(X * a, 3.0, window=7, branches=1, C=4e-6)
    assert np.array_equal(r2[2], r1[2] * np.float32(16.0))
    k1 = [(c["triple"], c["label"], c["n_pix"], c["peak_y"], c["peak_x"]) for c in r1[0]]
    k2 = [(c["triple"], c["label"], c["n_pix"], c["peak_y"], c["peak_x"]) for c in r2[0]]
    assert k1 == k2


def test_candidate_capacity_truncation():
    X = structured_stack(101, 8, 100, 500)
    full = run_gpu(X, 2.0, window=5, branches=1)
    assert len(full[0]) > 5
    part = run_gpu(X, 2.0, window=5, branches=1, cand_cap=3)
    assert part[5] == -4
    assert part[1]["n_cand"] == len(full[0])
    assert part[0] == full[0][:3]


def test_internal_capacity_flag():
    X = structured_stack(102, 8, 100, 500)
    cands, stats, q, eta, used, rc = run_gpu(X, 1.0, window=5, branches=1, max_segments=4)
    assert rc == -4
    assert all(f & 2 for f in stats["flags"])


@pytest.mark.parametrize("w,dt", [(9, "f16"), (7, "f32")])
def test_crop_interior_bitwise(w, dt):
    """q at the interior cells of a crop whose origin is a multiple of 16 is
    the full image's bit for bit (the window sums follow absolute 8-aligned
    blocks), which the crop error report relies on."""
    X = structured_stack(91, 6, 300, 700)
    _, _, q_full, _, _, _ = run_gpu(X, 5.0, dtype=dt, window=w)
    h = w // 2
    for oy, ox in ((16, 32), (48, 240), (0, 464)):
        C = np.ascontiguousarray(X[:, oy:oy + 200, ox:ox + 208])
        _, _, q_crop, _, _, _ = run_gpu(C, 5.0, dtype=dt, window=w)
        a = q_crop[:, h:-h, h:-h]
        b = q_full[:, oy + h:oy + 200 - h, ox + h:ox + 208 - h]
        assert a.tobytes() == b.tobytes(), (oy, ox)


@pytest.mark.parametrize("n,H,W,window,branches,dtype,sigma_est,harm", [
    (12, 48, 300, 5, 7, "f32", 0, 0),     # n' = 10, all three branches
    (32, 40, 200, 5, 4, "f32", 0, 0),     # n' = 30 (one round of four step groups)
    (26, 21, 77, 3, 5, "f32", 0, 2),      # n' = 24, harmonic sum, H*W not a multiple of 4
    (33, 30, 96, 7, 4, "f16", 1, 0),      # n' = 31 (odd), median/MAD
    (34, 40, 260, 3, 4, "f32", 0, 0),     # n' = 32, per-pixel branch alone
    (66, 30, 130, 5, 5, "f32", 1, 3),     # n' = 64, median/MAD, harmonic sum
    (22, 37, 250, 7, 6, "f16", 0, 0),     # FP16 storage
    (67, 20, 70, 3, 5, "f32", 0, 0),      # n' = 65
    (128, 16, 90, 3, 4, "f32", 0, 0),     # n' = 126, the longest serving request
    (129, 13, 37, 1, 4, "f32", 0, 2),     # n' = 127 (odd), harmonic sum, H*W not a multiple of 4
    (34, 300, 700, 9, 5, "f32", 0, 0),    # 3282 tiles of 64 pixels
    (34, 300, 700, 9, 5, "bf16", 1, 0),   # median/MAD of eta on a large map
])
def test_per_pixel_frequency_branch(n, H, W, window, branches, dtype, sigma_est, harm):
    """Per-pixel spectra (Eq. (10) per cell) against the oracle element by
    element: eta within 1e-5 eta, its mean and spread within 1e-6, the
    candidates by component."""
    rng = np.random.default_rng(n * 7 + H)
    X = structured_stack(n + H, n, H, W)
    y0, x0 = int(rng.integers(min(5, H - 4), H - 3)), int(rng.integers(5, W - 8))
    X[1::5, y0:y0 + 3, x0:x0 + 3] += 9.0
    tau = 4.0
    cands, stats, q, eta, used, rc = run_gpu(X, tau, dtype=dtype, window=window, branches=branches,
                                             sigma_est=sigma_est, harm=harm, tile=16, eta_px=True)
    assert rc == 0
    out = ref.detect(used, tau=tau, window=window, branches=branches, sigma_est=sigma_est, harm=harm, tile=16,
                     keep_maps=True)
    assert stats["ran"] & ref.FREQ_PIXEL
    if branches & ref.IMAGE:
        check_maps(q, out["q"])
    check_eta(stats["eta_px_map"], out["eta_px"])
    assert stats["eta_px_mu"] == pytest.approx(out["eta_px_mu"], rel=1e-6)
    assert stats["eta_px_sigma"] == pytest.approx(out["eta_px_sigma"], rel=1e-6)
    check_candidates(cands, out, tau)
    px = [c for c in cands if c["branch"] == ref.FREQ_PIXEL]
    assert px and all(c["triple"] == -1 for c in px)
    assert stats["n_freq_px_cand"] == len(px)


def test_per_pixel_branch_needs_four_triples():
    """With n' = 3 the frequency branches do not run, and say so."""
    X = structured_stack(5, 5, 20, 30)
    cands, stats, q, eta, used, rc = run_gpu(X, 3.0, window=3, branches=7, eta_px=True)
    assert rc == 0
    assert stats["ran"] == ref.IMAGE
    assert not [c for c in cands if c["branch"] != ref.IMAGE]


def test_per_pixel_series_limit_is_an_error():
    """A harmonic sum over a per-pixel series longer than the kernel's LDS
    table allows is refused, never skipped."""
    from paper_2509_21754_amd import FitrigError

    X = np.random.default_rng(7).normal(size=(452, 4, 8)).astype(np.float32)
    with pytest.raises(FitrigError):
        run_gpu(X, 3.0, window=3, branches=4, harm=2, with_maps=False)
    # the same length with h = max runs
    cands, stats, *_ = run_gpu(X, 3.0, window=3, branches=4, harm=0, with_maps=False)
    assert stats["ran"] == ref.FREQ_PIXEL


@pytest.mark.parametrize("mode,branches", [(0, 2), (1, 2), (0, 4)])
def test_index_map_written_without_image_branch(mode, branches):
    """The index map is written whenever it is requested."""
    X = structured_stack(17, 8, 40, 96)
    cands, stats, q, eta, used, rc = run_gpu(X, 3.0, window=5, mode=mode, tile=8, branches=branches)
    want = ref.index_maps(used, mode=mode, window=5, tile=8)
    check_maps(q, want)


def test_async_call_on_a_stream():
    """A call on a non-null stream returns at once; after the stream is
    synchronised its outputs equal the synchronous call's."""
    import ctypes

    from paper_2509_21754_amd import Context

    X = structured_stack(23, 12, 96, 400)
    t = torch.from_numpy(X).cuda()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with Context(window=7) as ctx:
        sync = ctx.detect(t, 4.0, as_dicts=False)
        b = ctx._buffers(1 << 16, 10)
        rc = ctx.enqueue(t, 4.0, b, 1 << 16, None, None, None, s)
        assert rc == 0
        s.synchronize()
        n = b["n"].value
        got = np.ctypeslib.as_array((ctypes.c_uint8 * (n * 72)).from_address(ctypes.addressof(b["cand"]))).copy()
        assert n == len(sync[0]) and got.tobytes() == sync[0].tobytes()
        assert list(b["mu"][:10]) == sync[1]["mu"] and b["st"].status == 0


def test_graph_capture_replays_bitwise():
    """The MEAN_STD image + frequency path captured into a HIP graph: three
    replays, with eager work and synchronisations between them, each equal
    byte for byte to the eager call."""
    import ctypes

    from paper_2509_21754_amd import Context

    X = structured_stack(29, 14, 150, 700)
    for k in range(2, 14, 4):
        X[k, 60:67, 300:307] += 30.0
    t = torch.from_numpy(X).cuda()
    qmap = torch.zeros((12, 150, 700), device="cuda")
    torch.cuda.synchronize()
    with Context(window=7, max_pixels=150 * 700, max_snap=14) as ctx:
        ref_c, ref_st, _ = ctx.detect(t, 4.0, index_map=qmap, as_dicts=False)
        q_ref = qmap.clone()
        assert len(ref_c) > 0
        s = torch.cuda.Stream()
        b = ctx._buffers(1 << 16, 12)
        with torch.cuda.stream(s):
            assert ctx.enqueue(t, 4.0, b, 1 << 16, qmap, None, None, s) == 0   # warm, outside the graph
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            assert ctx.enqueue(t, 4.0, b, 1 << 16, qmap, None, None, s) == 0
        for rep in range(3):
            qmap.fill_(float("nan"))
            b["n"].value = -1
            junk = (t[:3] * 2.0).sum()          # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            n = b["n"].value
            got = np.ctypeslib.as_array((ctypes.c_uint8 * (n * 72)).from_address(ctypes.addressof(b["cand"]))).copy()
            assert n == len(ref_c) and got.tobytes() == ref_c.tobytes(), rep
            assert torch.equal(qmap, q_ref), rep
            assert list(b["mu"][:12]) == ref_st["mu"] and list(b["sg"][:12]) == ref_st["sigma"], rep
            del junk
        del g
