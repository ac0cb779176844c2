"""Median/MAD spread at full image sizes, where the index pass writes the
bracket sample on its grid (the first cell of every 16-cell chunk in the
first row of every sampled band) instead of the hashed sample read from the
map. The library's location and spread of each checked triple must equal the
exact order statistics of its own q map, evaluated here with a partition in
the library's arithmetic: the median is the mean of the two middle values of
q, the MAD that of |q - median| rounded to FP32, sigma = 1.482602218505602 *
MAD (the robust reading of the spread of Eq. (8)). The q map itself is
compared with the FP64 oracle in the parity and full-size suites; this checks
the sample, the brackets, the gathering and the selection on sets of 2^28 and
2^29 cells."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

MAD_SCALE = 1.482602218505602


def exact_median_mad(q: np.ndarray):
    q = q.reshape(-1)
    n = q.size
    lo, hi = (n - 1) // 2, n // 2
    part = np.partition(q, [lo, hi])
    med = 0.5 * (float(part[lo]) + float(part[hi]))
    dev = np.abs(q.astype(np.float64) - med).astype(np.float32)
    dp = np.partition(dev, [lo, hi])
    return med, MAD_SCALE * (0.5 * (float(dp[lo]) + float(dp[hi])))


def run_mad(stack, window, tau, triples):
    from paper_2509_21754_amd import Context

    n, H, W = stack.shape
    qmap = torch.empty((n - 2, H, W), dtype=torch.float32, device="cuda")
    with Context(window=window, max_pixels=H * W, max_snap=n, sigma_est=1, branches=1) as ctx:
        cands, stats, rc = ctx.detect(stack, tau, index_map=qmap, cand_cap=1 << 18, as_dicts=False)
    torch.cuda.synchronize()
    assert rc == 0
    assert all(int(f) == 0 for f in stats["flags"])
    for s in triples:
        print(f"[mad fullsize] {H}x{W} triple {s}: exact order statistics", flush=True)
        med, sg = exact_median_mad(qmap[s].cpu().numpy())
        assert stats["mu"][s] == med, (s, stats["mu"][s], med)
        assert stats["sigma"][s] == sg, (s, stats["sigma"][s], sg)
    return stats


def test_median_mad_grid_sample_headline_stack():
    """The 16384^2 x 32 FP32 headline stack (window 9): every band sampled,
    67 column groups; three seeded triples checked."""
    import synth

    spec = synth.WORKLOADS["c2"]
    print("[mad fullsize] generating the 16384^2 x 32 stack", flush=True)
    stack = synth.make_stack(spec, device="cuda")
    torch.cuda.synchronize()
    triples = sorted(np.random.default_rng(2024).choice(spec.n - 2, size=3, replace=False).tolist())
    run_mad(stack, spec.window, spec.taus[0], triples)


def test_median_mad_grid_sample_strided_ragged():
    """32768 x 16387 (2^29 cells per set): every second band sampled, and a
    last column group of 19 cells (two sample chunks)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    H, W = 32768, 16387
    stack = torch.randn((3, H, W), generator=g, device="cuda", dtype=torch.float32) + 3.0
    stack[1, 1000:1040, 5000:5040] += 25.0
    run_mad(stack, 5, 8.0, [0])


def test_median_mad_grid_sample_defeated():
    """Window 1 (q is pointwise): a pulse on every cell of the sample grid
    (rows and columns that are multiples of 16) makes every sampled q an
    outlier, so the brackets from the sample miss the middle ranks and the
    fallback selections run; the result must still be the exact order
    statistics. (tau is far above every z: only the spread is checked.)"""
    g = torch.Generator(device="cuda")
    g.manual_seed(91)
    H = W = 16384
    stack = torch.randn((3, H, W), generator=g, device="cuda", dtype=torch.float32) + 3.0
    stack[1, ::16, ::16] += 50.0
    run_mad(stack, 1, 1e9, [0])


@pytest.mark.parametrize("window", [1, 3])
def test_median_mad_gathered_ties(window):
    """A 4096^2 set (gathered selection from a hashed sample) whose q takes
    few distinct values: the bracket bounds can be one key, so every digit
    starts known, and the upper middle value lies in the same key or past
    the histogram; the result must still be the exact order statistics."""
    g = torch.Generator(device="cuda")
    g.manual_seed(5 + window)
    H = W = 4096
    stack = torch.randint(1, 4, (3, H, W), generator=g, device="cuda").to(torch.float32)
    run_mad(stack, window, 1e9, [0])
