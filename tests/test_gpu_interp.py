"""GPU tests of sub-cell peak localisation (fitrig_interp_peaks through the
C ABI) against the FP64 oracle in oracle/interp.py."""
import numpy as np
import pytest

from oracle import interp as I
from oracle import ref
from parity import structured_stack

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

METHODS = (I.BILINEAR, I.BICUBIC, I.SPLINE, I.MAKIMA)


def _gpu(m, peaks, method, sub):
    from paper_2509_21754_amd import interp_peaks

    t = torch.from_numpy(np.ascontiguousarray(m, dtype=np.float32)).cuda()
    out = interp_peaks(t, peaks, method=method, sub=sub)
    torch.cuda.synchronize()
    return out


def _check(m, peaks, method, sub, out):
    """The GPU's grid point holds the oracle's maximum (to rounding); where
    the oracle's maximum is unique beyond rounding the positions are equal."""
    m64 = np.asarray(m, dtype=np.float32).astype(np.float64)
    for (py, px), (gy, gx, gv) in zip(peaks, out):
        V = I.surface(m64, py, px, method, sub)
        a = int(round((gy - py) * sub)) + sub
        b = int(round((gx - px) * sub)) + sub
        assert 0 <= a <= 2 * sub and 0 <= b <= 2 * sub
        assert (gy, gx) == (py + (a - sub) / sub, px + (b - sub) / sub)
        vmax = V.max()
        tol = 1e-9 * (1.0 + abs(vmax))
        assert V[a, b] >= vmax - tol, (py, px, method)
        assert gv == pytest.approx(V[a, b], rel=1e-9, abs=1e-9)
        second = np.sort(V.ravel())[-2]
        if second < vmax - tol:
            oy, ox, _ = I.interp_peak(m64, py, px, method, sub)
            assert (gy, gx) == (oy, ox)


@pytest.mark.parametrize("method", METHODS)
def test_interp_quadratic_peak_exact(method):
    yy, xx = np.mgrid[0:24, 0:20].astype(np.float64)
    for y0, x0 in ((10.25, 7.5), (9.8125, 8.0625), (12.0, 3.0)):
        m = (100.0 - 1.5 * (yy - y0) ** 2 - 0.75 * (xx - x0) ** 2).astype(np.float32)
        peaks = [(int(round(y0)), int(round(x0)))]
        out = _gpu(m, peaks, method, 16)
        _check(m, peaks, method, 16, out)
        if method in (I.BICUBIC, I.SPLINE):
            assert (out[0, 0], out[0, 1]) == (y0, x0)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("sub", [1, 5, 16])
def test_interp_random_maps(method, sub):
    rng = np.random.default_rng(100 + 7 * method + sub)
    H, W = 37, 53
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    m = rng.normal(size=(H, W)) * 0.05
    for _ in range(12):
        cy, cx = rng.uniform(-1, H), rng.uniform(-1, W)
        m += rng.uniform(1, 5) * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * rng.uniform(0.6, 2.5) ** 2))
    m = m.astype(np.float32)
    pad = np.pad(m, 1, constant_values=-np.inf)
    nb = np.stack([pad[1 + dy:1 + dy + H, 1 + dx:1 + dx + W] for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                   if (dy, dx) != (0, 0)])
    peaks = [tuple(map(int, p)) for p in np.argwhere(m > nb.max(axis=0))]
    peaks += [(0, 0), (H - 1, W - 1), (0, W - 1), (H // 2, 0)]   # edges and corners
    out = _gpu(m, peaks, method, sub)
    assert out.shape == (len(peaks), 3)
    _check(m, peaks, method, sub, out)


def test_interp_fine_grid_and_empty():
    from paper_2509_21754_amd import interp_peaks

    rng = np.random.default_rng(5)
    m = rng.normal(size=(9, 11)).astype(np.float32)
    peaks = [(4, 5), (0, 10)]
    out = _gpu(m, peaks, I.SPLINE, 64)
    _check(m, peaks, I.SPLINE, 64, out)
    t = torch.from_numpy(m).cuda()
    assert interp_peaks(t, np.zeros((0, 2), np.int32)).shape == (0, 3)


def test_interp_on_eta_of_a_periodic_source():
    """Localise frequency-branch candidates on the library's eta map; the
    oracle localises on its own eta map of the same stack."""
    from paper_2509_21754_amd import Context, interp_peaks

    X = structured_stack(77, 34, 128, 192)
    for k in range(0, 34, 4):
        X[k, 70:77, 101:108] += 10.0
    tau = 3.0
    Ty, Tx = 128 // 16, 192 // 16
    eta = torch.zeros((Ty, Tx), dtype=torch.float32, device="cuda")
    with Context(window=5, branches=2, tile=16) as ctx:
        cands, stats, rc = ctx.detect(torch.from_numpy(X).cuda(), tau, eta_map=eta)
    assert rc == 0 and cands
    peaks = [(c["peak_y"], c["peak_x"]) for c in cands]
    out = interp_peaks(eta, peaks, method=I.SPLINE, sub=16)
    oeta = ref.detect(X.astype(np.float64), tau=tau, window=5, branches=ref.FREQ, tile=16)["eta"]
    for (py, px), (gy, gx, gv) in zip(peaks, out):
        oy, ox, ov = I.interp_peak(oeta, py, px, I.SPLINE, 16)
        assert abs(gy - oy) <= 1 / 16 and abs(gx - ox) <= 1 / 16
        assert gv == pytest.approx(ov, rel=1e-4)
