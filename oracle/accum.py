"""Snapshot accumulation for short sampling periods (CPU oracle).

TEST INFRASTRUCTURE ONLY (like ``ref.py``): used by the tests, never by the
GPU library or its binding; shares no code with it.

When the sampling period is very short, adjacent snapshots are nearly the
same and their differences nearly blank; the paper then applies the method to
sums of adjacent snapshots, combined until adjacent sums differ enough
(Sec. 3.3.2, Fig. accum: the combination is a plain sum). The paper gives no
criterion for "enough". The readings here:

* one factor K for the whole stack: accumulated snapshot
  Y_j = sum_{k = jK}^{jK + K - 1} X_k for j = 0 .. P - 1, P = floor(n / K)
  (the last n - PK snapshots are dropped), so the accumulated series stays
  uniformly sampled (period K T_s), which the frequency branch needs;
* the contrast of adjacent sums j, j + 1 is the relative L1 difference
  c_j = sum_p |Y_{j+1}(p) - Y_j(p)| / sum_p |Y_j(p)| over all pixels p, and
  the contrast of a factor is C(K) = median_j c_j over the P - 1 pairs (the
  mean of the two middle values for an even count);
* the automatic factor is the smallest K in 1 .. k_max with P(K) >= 3 (the
  method needs three snapshots) and C(K) >= gamma; when none reaches gamma,
  the largest such K with P(K) >= 3.

The sums are formed in FP32, adding the snapshots in frame order (the
precision of the accumulated stack the method then reads, and the precision
in which the contrast decides K); the contrast reductions are FP64.
``accumulate_exact`` gives the FP64 sums for the error bound.
"""
from __future__ import annotations

import numpy as np


def accumulate(X, K: int) -> np.ndarray:
    """[P][H][W] float32: sums of K consecutive snapshots, in frame order, in FP32."""
    X = np.asarray(X)
    n = X.shape[0]
    if K < 1:
        raise ValueError("K must be >= 1")
    P = n // K
    Y = np.zeros((P,) + X.shape[1:], dtype=np.float32)
    for j in range(P):
        acc = X[j * K].astype(np.float32)
        for k in range(1, K):
            acc = acc + X[j * K + k].astype(np.float32)  # one FP32 rounding per addition
        Y[j] = acc
    return Y


def accumulate_exact(X, K: int) -> np.ndarray:
    """[P][H][W] float64: the same sums without rounding (for error bounds)."""
    X = np.asarray(X, dtype=np.float64)
    P = X.shape[0] // K
    return X[:P * K].reshape((P, K) + X.shape[1:]).sum(axis=1)


def pair_sums(Y) -> np.ndarray:
    """[P - 1][2] float64: (sum |Y_{j+1} - Y_j|, sum |Y_j|) for each adjacent pair,
    the differences taken in the precision of Y."""
    Y = np.asarray(Y)
    out = np.zeros((max(Y.shape[0] - 1, 0), 2))
    for j in range(Y.shape[0] - 1):
        d = np.abs(Y[j + 1] - Y[j])
        out[j, 0] = d.astype(np.float64).sum()
        out[j, 1] = np.abs(Y[j]).astype(np.float64).sum()
    return out


def contrast(X, K: int) -> float:
    """C(K): median over adjacent pairs of the relative L1 difference (NaN when
    there are fewer than two accumulated snapshots)."""
    Y = accumulate(X, K)
    if Y.shape[0] < 2:
        return float("nan")
    ps = pair_sums(Y)
    c = np.where(ps[:, 1] > 0, ps[:, 0] / np.where(ps[:, 1] > 0, ps[:, 1], 1.0), np.inf)
    c = np.where((ps[:, 0] == 0) & (ps[:, 1] == 0), 0.0, c)
    c = np.sort(c)
    m = len(c)
    return float(c[m // 2]) if m % 2 else float(0.5 * (c[m // 2 - 1] + c[m // 2]))


def accum_factor(X, gamma: float, k_max: int):
    """(K, [C(1), ..., C(k_max)]): the automatic accumulation factor."""
    n = np.asarray(X).shape[0]
    cs = [contrast(X, K) for K in range(1, k_max + 1)]
    eligible = [K for K in range(1, k_max + 1) if n // K >= 3]
    if not eligible:
        raise ValueError("fewer than three snapshots")
    for K in eligible:
        if cs[K - 1] >= gamma:
            return K, cs
    return eligible[-1], cs
