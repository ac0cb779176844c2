"""Pins of the snapshot-accumulation oracle (oracle/accum.py): closed forms
for ramps and constant stacks, conservation of the summed signal, the
identity at K = 1, brute force on tiny stacks, and the choice of the factor.
The paper gives no accumulation criterion (Sec. 3.3.2), so the criterion
itself is a reading and parity with the paper's own choice is unpinned."""
import numpy as np
import pytest

from oracle import accum


def test_k1_is_the_identity_and_sums_are_conserved():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(11, 5, 7)).astype(np.float32)
    assert np.array_equal(accum.accumulate(X, 1), X)
    for K in (2, 3, 5):
        Y = accum.accumulate_exact(X, K)
        P = 11 // K
        assert Y.shape == (P, 5, 7)
        np.testing.assert_allclose(Y.sum(axis=0), X[:P * K].astype(np.float64).sum(axis=0), rtol=1e-12, atol=1e-12)
        # FP32 sums within the bound of K - 1 roundings of the running sum
        Yf = accum.accumulate(X, K).astype(np.float64)
        bound = (K - 1) * 2.0 ** -24 * np.abs(X[:P * K].astype(np.float64)).reshape((P, K, 5, 7)).sum(axis=1)
        assert np.all(np.abs(Yf - Y) <= bound + 1e-30)


def test_brute_force_pair_sums_and_median():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(9, 3, 4)).astype(np.float32)
    for K in (1, 2, 3, 4):
        P = 9 // K
        Y = [[[0.0] * 4 for _ in range(3)] for _ in range(P)]
        for j in range(P):
            for y in range(3):
                for x in range(4):
                    a = np.float32(X[j * K, y, x])
                    for k in range(1, K):
                        a = np.float32(a + np.float32(X[j * K + k, y, x]))
                    Y[j][y][x] = a
        cs = []
        for j in range(P - 1):
            num = sum(abs(float(np.float32(Y[j + 1][y][x] - Y[j][y][x]))) for y in range(3) for x in range(4))
            den = sum(abs(float(Y[j][y][x])) for y in range(3) for x in range(4))
            cs.append(num / den)
        cs.sort()
        m = len(cs)
        med = cs[m // 2] if m % 2 else 0.5 * (cs[m // 2 - 1] + cs[m // 2])
        assert accum.contrast(X, K) == pytest.approx(med, rel=1e-13)


def test_ramp_closed_form():
    # X_k = a + b k on every pixel (a, b > 0): Y_{j+1} - Y_j = b K^2 and
    # Y_j = K a + b (K^2 j + K (K - 1) / 2), so c_j = b K / (a + b (K j + (K - 1) / 2))
    a, b, n = 64.0, 1.0, 24
    X = (a + b * np.arange(n, dtype=np.float64))[:, None, None] * np.ones((1, 2, 3))
    X = X.astype(np.float32)
    for K in (1, 2, 3, 4, 6):
        P = n // K
        c = sorted(b * K / (a + b * (K * j + (K - 1) / 2.0)) for j in range(P - 1))
        m = len(c)
        med = c[m // 2] if m % 2 else 0.5 * (c[m // 2 - 1] + c[m // 2])
        assert accum.contrast(X, K) == pytest.approx(med, rel=1e-12)
    # the contrast grows with K here, so the factor is the first K reaching gamma
    cs = [accum.contrast(X, K) for K in range(1, 7)]
    assert all(x < y for x, y in zip(cs, cs[1:]))
    K, got = accum.accum_factor(X, 0.05, 6)
    assert K == min(k for k in range(1, 7) if cs[k - 1] >= 0.05) and got == cs


def test_constant_stack_never_reaches_gamma():
    X = np.full((12, 4, 4), 3.0, dtype=np.float32)
    for K in range(1, 5):
        assert accum.contrast(X, K) == 0.0
    K, _ = accum.accum_factor(X, 1e-3, 8)
    assert K == 4          # the largest K that still leaves three accumulated snapshots


def test_noise_needs_no_accumulation():
    # independent noise: adjacent snapshots already differ by ~ sqrt(2) of their size
    X = np.random.default_rng(2).normal(size=(16, 64, 64)).astype(np.float32)
    assert accum.contrast(X, 1) == pytest.approx(np.sqrt(2.0), rel=0.05)
    assert accum.accum_factor(X, 0.5, 8)[0] == 1
