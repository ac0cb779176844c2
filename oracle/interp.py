"""Sub-cell peak localisation by interpolation (FP64 CPU oracle).

TEST INFRASTRUCTURE ONLY (like ``ref.py``): used by the tests and the smoke
check, never by the GPU library or its binding; shares no code with it.

The paper localises a source inside the selected tiles by interpolating the
tile values (the spectrum matrix eta) with a bilinear, spline, bicubic or
Makima cubic interpolant and taking the position of the interpolated maximum
(Sec. 2.4.2, applied with a spline in Sec. 3.1). The paper gives no
neighbourhood, grid or end conditions; the readings here:

* the 5 x 5 cells centred on the peak cell, cell indices clamped into the map
  (edge values repeated);
* a tensor-product interpolant: each of the 5 rows is interpolated along x,
  then the 5 row values along y;
* the surface evaluated at peak + (a, b) / sub for a, b = -sub .. sub; the
  reported position is the grid point of the largest value, ties to the
  smallest a, then the smallest b;
* methods on unit-spaced nodes f[0..4] at t in [0, 4]:
  bilinear - straight lines between nodes;
  bicubic  - cubic convolution with the Keys kernel, a = -1/2;
  spline   - the cubic spline through the nodes with not-a-knot end
             conditions (third derivative continuous at nodes 1 and 3);
  makima   - the modified Akima piecewise cubic: node slope
             (w1 d[i-1] + w2 d[i]) / (w1 + w2) with
             w1 = |d[i+1] - d[i]| + |d[i+1] + d[i]| / 2,
             w2 = |d[i-1] - d[i-2]| + |d[i-1] + d[i-2]| / 2,
             d the interval slopes, extended linearly by two intervals on each
             side; zero weights (all four slopes zero) give slope 0.
"""
from __future__ import annotations

import math

import numpy as np

BILINEAR, BICUBIC, SPLINE, MAKIMA = 0, 1, 2, 3
RADIUS = 2
N = 2 * RADIUS + 1


def keys_weight(s: float, a: float = -0.5) -> float:
    """Keys' cubic convolution kernel."""
    s = abs(s)
    if s <= 1.0:
        return (a + 2.0) * s ** 3 - (a + 3.0) * s ** 2 + 1.0
    if s < 2.0:
        return a * s ** 3 - 5.0 * a * s ** 2 + 8.0 * a * s - 4.0 * a
    return 0.0


def _interval(t: float) -> int:
    return min(max(int(math.floor(t)), 0), N - 2)


def _hermite(f0, f1, d0, d1, u):
    """Cubic Hermite on a unit interval at u in [0, 1]."""
    h00 = 2 * u ** 3 - 3 * u ** 2 + 1
    h10 = u ** 3 - 2 * u ** 2 + u
    h01 = -2 * u ** 3 + 3 * u ** 2
    h11 = u ** 3 - u ** 2
    return h00 * f0 + h10 * d0 + h01 * f1 + h11 * d1


def spline_second_derivatives(f) -> np.ndarray:
    """Not-a-knot cubic spline on unit-spaced nodes: the node second
    derivatives M from continuity of the second derivative at the interior
    nodes plus equal third derivatives on the first two and last two intervals."""
    n = len(f)
    A = np.zeros((n, n))
    r = np.zeros(n)
    A[0, 0:3] = (1.0, -2.0, 1.0)
    for i in range(1, n - 1):
        A[i, i - 1:i + 2] = (1.0, 4.0, 1.0)
        r[i] = 6.0 * (f[i - 1] - 2.0 * f[i] + f[i + 1])
    A[n - 1, n - 3:n] = (1.0, -2.0, 1.0)
    return np.linalg.solve(A, r)


def makima_slopes(f) -> np.ndarray:
    n = len(f)
    d = [f[i + 1] - f[i] for i in range(n - 1)]
    # two extra intervals on each side, extended linearly
    left1 = 2.0 * d[0] - d[1]
    left2 = 2.0 * left1 - d[0]
    right1 = 2.0 * d[-1] - d[-2]
    right2 = 2.0 * right1 - d[-1]
    m = [left2, left1] + d + [right1, right2]   # m[k + 2] = d[k]
    out = np.zeros(n)
    for i in range(n):
        dm2, dm1, d0, dp1 = m[i], m[i + 1], m[i + 2], m[i + 3]   # d[i-2], d[i-1], d[i], d[i+1]
        w1 = abs(dp1 - d0) + abs(dp1 + d0) / 2.0
        w2 = abs(dm1 - dm2) + abs(dm1 + dm2) / 2.0
        out[i] = 0.0 if w1 + w2 == 0.0 else (w1 * dm1 + w2 * d0) / (w1 + w2)
    return out


def interp1(f, t: float, method: int) -> float:
    """Value at t in [0, N-1] of the interpolant through f[0..N-1] (unit spacing)."""
    f = [float(v) for v in f]
    i = _interval(t)
    u = t - i
    if method == BILINEAR:
        return (1.0 - u) * f[i] + u * f[i + 1]
    if method == BICUBIC:
        s = 0.0
        for k in range(i - 1, i + 3):
            kk = min(max(k, 0), N - 1)
            s += keys_weight(t - k) * f[kk]
        return s
    if method == SPLINE:
        M = spline_second_derivatives(f)
        return (M[i] * (1.0 - u) ** 3 / 6.0 + M[i + 1] * u ** 3 / 6.0
                + (f[i] - M[i] / 6.0) * (1.0 - u) + (f[i + 1] - M[i + 1] / 6.0) * u)
    if method == MAKIMA:
        dd = makima_slopes(f)
        return _hermite(f[i], f[i + 1], dd[i], dd[i + 1], u)
    raise ValueError(method)


def neighbourhood(m: np.ndarray, py: int, px: int) -> np.ndarray:
    H, W = m.shape
    F = np.empty((N, N))
    for r in range(N):
        for c in range(N):
            y = min(max(py - RADIUS + r, 0), H - 1)
            x = min(max(px - RADIUS + c, 0), W - 1)
            F[r, c] = m[y, x]
    return F


def surface(m: np.ndarray, py: int, px: int, method: int, sub: int) -> np.ndarray:
    """Interpolated values at peak + (a, b) / sub, a and b from -sub to sub."""
    F = neighbourhood(np.asarray(m, dtype=np.float64), py, px)
    G = np.empty((N, 2 * sub + 1))
    for bi in range(2 * sub + 1):
        t = RADIUS + (bi - sub) / sub
        for r in range(N):
            G[r, bi] = interp1(F[r], t, method)
    V = np.empty((2 * sub + 1, 2 * sub + 1))
    for ai in range(2 * sub + 1):
        t = RADIUS + (ai - sub) / sub
        for bi in range(2 * sub + 1):
            V[ai, bi] = interp1(G[:, bi], t, method)
    return V


def interp_peak(m: np.ndarray, py: int, px: int, method: int, sub: int = 16):
    """(y, x, value) of the interpolated maximum near peak cell (py, px)."""
    V = surface(m, py, px, method, sub)
    best = None
    for ai in range(2 * sub + 1):
        for bi in range(2 * sub + 1):
            if best is None or V[ai, bi] > best[0]:
                best = (V[ai, bi], ai, bi)
    v, ai, bi = best
    return py + (ai - sub) / sub, px + (bi - sub) / sub, v
