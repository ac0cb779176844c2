"""Snapshot accumulation on the GPU (fitrig_accumulate / fitrig_accum_factor,
through the C ABI) against the oracle (oracle/accum.py): the accumulated
stack bit for bit (FP32 sums in frame order, FP32/FP16/BF16 storage), the
contrasts C(K) and the chosen factor, and the whole path run on an
accumulated stack against the FP64 oracle on the same accumulated values."""
import numpy as np
import pytest

from oracle import accum, ref
from parity import check_candidates, check_maps, check_stats, structured_stack

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def _slow_stack(seed, n, H, W):
    """Noise plus a source whose flux changes slowly (a snapshot sampled far
    faster than its variation), scaled down so adjacent snapshots nearly agree."""
    rng = np.random.default_rng(seed)
    X = 0.001 * rng.normal(size=(n, H, W)) + 40.0
    t = np.arange(n)
    X[:, 10:40, 20:60] += (5.0 * np.sin(2 * np.pi * t / n))[:, None, None]
    return X.astype(np.float32)


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("K", [1, 2, 3, 7])
def test_accumulate_bitwise(dt, K):
    from paper_2509_21754_amd import accumulate

    X = structured_stack(70 + K, 23, 67, 301)
    t = torch.from_numpy(X).to(DT[dt]).cuda()
    used = t.float().cpu().numpy()
    Y = accumulate(t, K)
    torch.cuda.synchronize()
    assert Y.cpu().numpy().tobytes() == accum.accumulate(used, K).tobytes()


@pytest.mark.parametrize("make,gamma,kmax", [(_slow_stack, 0.004, 8), (_slow_stack, 0.002, 6),
                                             (lambda s, n, H, W: structured_stack(s, n, H, W), 0.5, 5)])
def test_accum_factor_matches_oracle(make, gamma, kmax):
    from paper_2509_21754_amd import accum_factor

    X = make(80, 40, 90, 130)
    t = torch.from_numpy(X).cuda()
    torch.cuda.synchronize()
    K, C = accum_factor(t, gamma, kmax)
    K_ref, C_ref = accum.accum_factor(X, gamma, kmax)
    for k in range(kmax):
        if np.isnan(C_ref[k]):
            assert np.isnan(C[k])
        else:
            assert C[k] == pytest.approx(C_ref[k], rel=1e-12), k
    near = [k for k in range(kmax) if abs(C_ref[k] - gamma) <= 1e-9 * max(gamma, 1e-300)]
    if not near:
        assert K == K_ref, (K, K_ref, C_ref)


def test_accum_factor_picks_more_than_one_for_slow_variation():
    from paper_2509_21754_amd import accum_factor

    X = _slow_stack(81, 48, 64, 96)
    K, C = accum_factor(torch.from_numpy(X).cuda(), 0.008, 8)
    assert K == 5 and C[0] < 0.008 <= C[K - 1]


@pytest.mark.parametrize("K", [2, 4])
def test_path_on_accumulated_stack(K):
    from paper_2509_21754_amd import Context, accumulate

    X = structured_stack(90 + K, 28, 96, 300, pulse_amp=20.0)
    t = torch.from_numpy(X).cuda()
    Y = accumulate(t, K)
    n2 = Y.shape[0]
    qmap = torch.empty((n2 - 2, 96, 300), device="cuda")
    with Context(window=7, tile=16) as ctx:
        cands, stats, rc = ctx.detect(Y, 4.0, index_map=qmap)
    torch.cuda.synchronize()
    Yr = accum.accumulate(X, K)
    assert Y.cpu().numpy().tobytes() == Yr.tobytes()
    out = ref.detect(Yr.astype(np.float64), tau=4.0, window=7, tile=16)
    check_maps(qmap.cpu().numpy(), out["q"])
    check_stats(stats["mu"], stats["sigma"], out["mu"], out["sigma"], out["flags"])
    check_candidates(cands, out, 4.0)


def test_accum_argument_errors():
    from paper_2509_21754_amd import FitrigError, accum_factor, accumulate

    t = torch.zeros((5, 8, 8), device="cuda")
    with pytest.raises(FitrigError):
        accumulate(t, 6)
    with pytest.raises(FitrigError):
        accumulate(t, 0)
    with pytest.raises(FitrigError):
        accum_factor(t, -1.0, 3)
    with pytest.raises(FitrigError):
        accum_factor(t[:2].contiguous(), 0.1, 3)
