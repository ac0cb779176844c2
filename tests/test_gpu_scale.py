"""GPU parity at the full 16384 x 16384 x 32 FP32 size (window 9, tau 6), in
the launch configuration the benchmark times, on outputs the FP64 oracle can
compute one by one:

* q at seeded sampled cells (image corners, edges, band and column-group
  seams, random interior cells), from a crop of the stack that holds each
  cell's clipped window;
* per-triple mean and std of q against a two-pass FP64 evaluation of the
  library's own q map (the spread stage at full size);
* for three seeded triples, the oracle's whole q map (from the triple's three
  frames): its mean and std against the library's, and every candidate of
  the triple against the oracle's components built with the oracle's own
  mean and std;
* a seeded sample of candidates of other triples: the oracle's component
  around the candidate's peak, built from oracle q over the candidate's box
  grown by two cells, with the library's mean and std."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import ref
from parity import CENTROID_TOL, MAP_ATOL_REL_MEAN, MAP_RTOL, STAT_RTOL, Z_BAND, check_components

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

H = W = 16384
N = 32
WIN = 9
TAU = 6.0
HALO = WIN // 2


@pytest.fixture(scope="module")
def c2_run():
    import synth
    from paper_2509_21754_amd import Context

    spec = synth.WORKLOADS["c2"]
    assert (spec.H, spec.W, spec.n, spec.window) == (H, W, N, WIN)
    print("[fullsize] generating the 16384^2 x 32 stack", flush=True)
    stack = synth.make_stack(spec, device="cuda")
    torch.cuda.synchronize()
    qmap = torch.empty((N - 2, H, W), dtype=torch.float32, device="cuda")
    with Context(window=WIN, max_pixels=H * W, max_snap=N) as ctx:
        cands, stats, rc = ctx.detect(stack, TAU, index_map=qmap, as_dicts=False)
        cands2, stats2, rc2 = ctx.detect(stack, TAU, as_dicts=False)   # without the map, as timed
    torch.cuda.synchronize()
    print(f"[fullsize] {len(cands)} candidates", flush=True)
    yield stack, qmap, cands, stats, rc, cands2, stats2, rc2
    del stack, qmap
    torch.cuda.empty_cache()


ORACLE_TRIPLES = (0, 13, 29)


@pytest.fixture(scope="module")
def c2_oracle(c2_run):
    """Oracle q, mean and std of whole triples (from their three frames)."""
    stack = c2_run[0]
    res = {}
    for s in ORACLE_TRIPLES:
        print(f"[fullsize] oracle on triple {s}", flush=True)
        X3 = stack[s:s + 3].cpu().numpy()
        q = ref.index_maps(X3, window=WIN)[0]
        del X3
        mu, sig = ref.spread(q)
        res[s] = (q, mu, sig)
    yield res


def test_fullsize_spread_against_oracle(c2_run, c2_oracle):
    stats = c2_run[3]
    for s, (_, mu, sig) in c2_oracle.items():
        assert stats["mu"][s] == pytest.approx(mu, rel=STAT_RTOL), s
        assert stats["sigma"][s] == pytest.approx(sig, rel=STAT_RTOL), s


def test_fullsize_candidates_against_oracle(c2_run, c2_oracle):
    from paper_2509_21754_amd.fitrig import _rec_dict

    cands = c2_run[2]
    total = 0
    for s, (q, mu, sig) in c2_oracle.items():
        g = [_rec_dict(c) for c in cands if c["branch"] == 1 and c["triple"] == s]
        r = ref.components(q, mu, sig, TAU)
        for c in r:
            c.update(branch=1, triple=s)
        total += check_components(g, r, q, mu, sig, TAU, where=f"triple {s}")
    assert total > 0


def _crop(stack, s, ya, yb, xa, xb):
    """Frames s..s+2, rows [ya, yb) and columns [xa, xb) as float32 numpy."""
    return stack[s:s + 3, ya:yb, xa:xb].float().cpu().numpy()


def _q_region(stack, s, y0, y1, x0, x1):
    """Oracle q over cells [y0, y1] x [x0, x1] of triple s (inclusive)."""
    ya, yb = max(0, y0 - HALO), min(H, y1 + HALO + 1)
    xa, xb = max(0, x0 - HALO), min(W, x1 + HALO + 1)
    X = _crop(stack, s, ya, yb, xa, xb)
    yy, xx = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
    cells = np.stack([np.zeros(yy.size, np.int64), (yy - ya).ravel(), (xx - xa).ravel()], 1)
    return ref.index_cells(X, cells, window=WIN).reshape(yy.shape)


def _sample_cells(seed):
    rng = np.random.default_rng(seed)
    ys = [0, 1, HALO, H - 1, H - 2, H - 1 - HALO, 15, 16, 17, 8191, 8192]
    xs = [0, 1, HALO, W - 1, W - 2, W - 1 - HALO, 239, 240, 241, 16319, 16320]
    cells = [(int(rng.integers(0, N - 2)), y, x) for y in ys for x in xs]
    cells += [(int(rng.integers(0, N - 2)), int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(600)]
    return cells


def test_fullsize_sampled_cells(c2_run):
    stack, qmap, *_ = c2_run
    cells = _sample_cells(2024)
    got = np.array([qmap[s, y, x].item() for s, y, x in cells])
    want = np.array([_q_region(stack, s, y, y, x, x)[0, 0] for s, y, x in cells])
    mean_q = [qmap[s].double().mean().item() for s in range(N - 2)]
    tol = MAP_RTOL * np.abs(want) + MAP_ATOL_REL_MEAN * np.array([mean_q[s] for s, _, _ in cells])
    bad = np.abs(got - want) > tol
    assert not bad.any(), list(zip(np.array(cells)[bad][:5].tolist(), got[bad][:5], want[bad][:5]))


def test_fullsize_spread(c2_run):
    _, qmap, _, stats, *_ = c2_run
    for s in range(N - 2):
        q = qmap[s].double()
        mu = q.mean().item()
        sig = (q - mu).pow(2).mean().sqrt().item()
        assert stats["mu"][s] == pytest.approx(mu, rel=STAT_RTOL)
        assert stats["sigma"][s] == pytest.approx(sig, rel=STAT_RTOL)


def test_fullsize_map_does_not_change_results(c2_run):
    _, _, cands, stats, rc, cands2, stats2, rc2 = c2_run
    assert rc == 0 and rc2 == 0
    assert cands.tobytes() == cands2.tobytes()
    assert stats["mu"] == stats2["mu"] and stats["sigma"] == stats2["sigma"]


def test_fullsize_sampled_candidates(c2_run):
    stack, _, cands, stats, *_ = c2_run
    img = cands[cands["branch"] == 1]
    assert len(img) > 0
    rng = np.random.default_rng(77)
    pick = rng.choice(len(img), size=min(120, len(img)), replace=False)
    checked = 0
    for i in pick:
        c = img[i]
        s = int(c["triple"])
        mu, sig = stats["mu"][s], stats["sigma"][s]
        y0, x0 = max(0, int(c["y0"]) - 2), max(0, int(c["x0"]) - 2)
        y1, x1 = min(H - 1, int(c["y1"]) + 2), min(W - 1, int(c["x1"]) + 2)
        q = _q_region(stack, s, y0, y1, x0, x1)
        z = (q - mu) / sig
        if np.any(np.abs(z - TAU) <= Z_BAND):
            continue
        comps, mask = ref.components(q, mu, sig, TAU, with_mask=True)
        py, px = int(c["peak_y"]) - y0, int(c["peak_x"]) - x0
        assert mask[py, px], (s, int(c["peak_y"]), int(c["peak_x"]))
        # the oracle component holding the peak: its label is the lowest
        # raster index of its cells in the region
        lab, _ = ndimage.label(mask, structure=np.ones((3, 3)))
        cells = np.flatnonzero(lab.ravel() == lab[py, px])
        d = next(d for d in comps if d["label"] == int(cells[0]))
        assert d["n_pix"] == int(c["n_pix"]) == len(cells)
        assert (d["y0"] + y0, d["x0"] + x0, d["y1"] + y0, d["x1"] + x0) == \
            (int(c["y0"]), int(c["x0"]), int(c["y1"]), int(c["x1"]))
        assert (d["peak_y"] + y0, d["peak_x"] + x0) == (int(c["peak_y"]), int(c["peak_x"]))
        assert abs(d["cy"] + y0 - float(c["cy"])) <= CENTROID_TOL
        assert abs(d["cx"] + x0 - float(c["cx"])) <= CENTROID_TOL
        checked += 1
    assert checked >= min(60, len(pick) // 2)
