"""FITrig FP64 CPU oracle: Python marshalling around ``fitrig_ref.c``.

TEST INFRASTRUCTURE ONLY. Imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark; never by the GPU library or its
binding. It shares no code with the HIP path.

The arithmetic lives in ``fitrig_ref.c`` (plain loops in double precision,
each step citing the paper). This module only converts arrays, calls those
loops in the paper's order and arranges the results:

* per-pixel / per-tile index q for every triple (Sec. 2.2.4 Eq. (2); the
  kernel form Eq. (6) of Sec. 2.3 is the same quantity);
* per-triple spread and selection z > tau with 8-connected components
  (Sec. 2.4.1 Eqs. (8)-(9));
* the image-frequency branch: tile cube over s, spectrum eta (Eq. (10)),
  z-score on eta and selection (Eqs. (11)-(12), Sec. 2.4.2);
* the same spectrum, z-score and selection per cell of the sliding index maps
  (the per-pixel form of Eq. (10); the paper transforms tiles).

Candidate order: image branch first (by triple, then label), then the
frequency branch (by label), then the per-pixel frequency branch (by label). Label = lowest row-major index of the component.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fitrig_ref.c")
# FITRIG_REF_LIB: another build of the same C source (the sanitizer test)
_LIB = os.environ.get("FITRIG_REF_LIB") or os.path.join(_HERE, "libfitrig_ref.so")

SLIDING, TILES = 0, 1
FREQ_PIXEL = 4
MEAN_STD, MEDIAN_MAD = 0, 1
IMAGE, FREQ = 1, 2
FLAG_SIGMA_ZERO = 1


class RefComp(ctypes.Structure):
    _fields_ = [
        ("label", ctypes.c_int64),
        ("n_pix", ctypes.c_int64),
        ("peak_y", ctypes.c_int64),
        ("peak_x", ctypes.c_int64),
        ("peak_z", ctypes.c_double),
        ("peak_q", ctypes.c_double),
        ("cy", ctypes.c_double),
        ("cx", ctypes.c_double),
        ("y0", ctypes.c_int64),
        ("x0", ctypes.c_int64),
        ("y1", ctypes.c_int64),
        ("x1", ctypes.c_int64),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP for the per-cell loops)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.ref_pixel_terms.argtypes = [vp, i32, i32, i64, i64, i32, i32, dbl, vp, vp]
        L.ref_set_threads.argtypes = [i32]
        L.ref_set_threads.restype = None
        L.ref_max_threads.argtypes = []
        L.ref_max_threads.restype = i32
        L.ref_normaliser.argtypes = [vp, i32, i64, dbl]
        L.ref_normaliser.restype = dbl
        L.ref_index_maps.argtypes = [vp, i32, i32, i64, i64, i32, i32, i32, i32, dbl, vp]
        L.ref_index_cells.argtypes = [vp, i32, i32, i64, i64, i32, i32, dbl, vp, i64, vp]
        L.ref_spread.argtypes = [vp, i64, i32, vp, vp]
        L.ref_components.argtypes = [vp, i64, i64, dbl, dbl, dbl, vp, vp, i64]
        L.ref_components.restype = i64
        L.ref_eta.argtypes = [vp, i32, i64, i32, vp]
        _lib = L
    return _lib


def _as_input(stack) -> tuple[np.ndarray, int]:
    """Decode the stack for the oracle: float32 is read as is (every float32
    is exact in double), float16 / bfloat16 are widened to float32 exactly,
    anything else becomes float64."""
    if hasattr(stack, "detach"):  # a torch tensor
        import torch

        t = stack.detach().cpu()
        if t.dtype in (torch.float16, torch.bfloat16):
            t = t.float()
        stack = t.numpy()
    a = np.asarray(stack)
    if a.dtype == np.float16:
        a = a.astype(np.float32)
    if a.dtype == np.float32:
        return np.ascontiguousarray(a), 1
    return np.ascontiguousarray(a, dtype=np.float64), 0


def pixel_terms(stack, s: int, *, r_signed: bool = False, C: float = 1e-6):
    """Delta and r planes of triple s (Eqs. (3)-(5))."""
    X, f32 = _as_input(stack)
    n, H, W = X.shape
    d = np.empty((H, W), np.float64)
    r = np.empty((H, W), np.float64)
    rc = lib().ref_pixel_terms(X.ctypes.data, f32, n, H, W, s, int(r_signed), C,
                               d.ctypes.data, r.ctypes.data)
    if rc != 0:
        raise ValueError(f"ref_pixel_terms failed ({rc})")
    return d, r


def normaliser(stack, C: float = 1e-6) -> float:
    """M = max(max over the whole stack, C) (Eq. (2))."""
    X, f32 = _as_input(stack)
    return float(lib().ref_normaliser(X.ctypes.data, f32, X.size, C))


def index_maps(stack, *, mode: int = SLIDING, window: int = 7, tile: int = 32,
               r_signed: bool = False, C: float = 1e-6) -> np.ndarray:
    """q maps [n-2][Ho][Wo] in float64 (sliding: H x W; tiles: ceil grid)."""
    X, f32 = _as_input(stack)
    n, H, W = X.shape
    if mode == SLIDING:
        Ho, Wo = H, W
    else:
        Ho, Wo = -(-H // tile), -(-W // tile)
    q = np.empty((n - 2, Ho, Wo), np.float64)
    rc = lib().ref_index_maps(X.ctypes.data, f32, n, H, W, mode, window, tile,
                              int(r_signed), C, q.ctypes.data)
    if rc != 0:
        raise ValueError(f"ref_index_maps failed ({rc})")
    return q


def index_cells(stack, cells, *, window: int = 7, r_signed: bool = False,
                C: float = 1e-6) -> np.ndarray:
    """Sliding-mode q at the given (s, y, x) cells."""
    X, f32 = _as_input(stack)
    n, H, W = X.shape
    c = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).reshape(-1, 3))
    out = np.empty(len(c), np.float64)
    rc = lib().ref_index_cells(X.ctypes.data, f32, n, H, W, window, int(r_signed), C,
                               c.ctypes.data, len(c), out.ctypes.data)
    if rc != 0:
        raise ValueError(f"ref_index_cells failed ({rc})")
    return out


def spread(q, estimator: int = MEAN_STD) -> tuple[float, float]:
    a = np.ascontiguousarray(np.asarray(q, dtype=np.float64).ravel())
    mu = ctypes.c_double()
    sig = ctypes.c_double()
    rc = lib().ref_spread(a.ctypes.data, a.size, estimator, ctypes.byref(mu), ctypes.byref(sig))
    if rc != 0:
        raise ValueError(f"ref_spread failed ({rc})")
    return mu.value, sig.value


def components(q2d, mu: float, sigma: float, tau: float, *, with_mask: bool = False):
    """8-connected components of {z > tau} on one 2-D map."""
    a = np.ascontiguousarray(np.asarray(q2d, dtype=np.float64))
    Ho, Wo = a.shape
    L = lib()
    mask = np.zeros((Ho, Wo), np.uint8)
    n = L.ref_components(a.ctypes.data, Ho, Wo, mu, sigma, tau, mask.ctypes.data, None, 0)
    if n < 0:
        raise ValueError("ref_components failed")
    buf = (RefComp * max(int(n), 1))()
    L.ref_components(a.ctypes.data, Ho, Wo, mu, sigma, tau, None, buf, n)
    comps = []
    for i in range(int(n)):
        c = buf[i]
        comps.append(dict(label=int(c.label), n_pix=int(c.n_pix), peak_y=int(c.peak_y),
                          peak_x=int(c.peak_x), peak_z=float(c.peak_z), peak_q=float(c.peak_q),
                          cy=float(c.cy), cx=float(c.cx), y0=int(c.y0), x0=int(c.x0),
                          y1=int(c.y1), x1=int(c.x1)))
    return (comps, mask.astype(bool)) if with_mask else comps


def eta(cube, harm: int = 0) -> np.ndarray:
    """eta over a tile cube [n'][Ty][Tx] (Eq. (10))."""
    c = np.ascontiguousarray(np.asarray(cube, dtype=np.float64))
    npr = c.shape[0]
    out = np.empty(c.shape[1:], np.float64)
    rc = lib().ref_eta(c.ctypes.data, npr, int(np.prod(c.shape[1:])), harm, out.ctypes.data)
    if rc != 0:
        raise ValueError(f"ref_eta failed ({rc})")
    return out


def detect(stack, *, tau: float = 6.0, mode: int = SLIDING, window: int = 7,
           tile: int = 32, branches: int = IMAGE | FREQ, sigma_est: int = MEAN_STD,
           harm: int = 0, r_signed: bool = False, C: float = 1e-6,
           keep_maps: bool = True) -> dict:
    """The whole path on the CPU in FP64, in the paper's order.

    Returns a dict with M, the q maps, per-triple mu / sigma / flags, the
    candidate list (dicts with ``branch`` and ``triple``), the tile cube and
    eta for the frequency branch (or None when n' < 4 or disabled).
    """
    X, _ = _as_input(stack)
    n = X.shape[0]
    if n < 3:
        raise ValueError("need at least three snapshots")
    M = normaliser(X, C)
    out: dict = {"M": M, "cands": [], "mu": [], "sigma": [], "flags": []}
    q = None
    if branches & IMAGE:
        q = index_maps(X, mode=mode, window=window, tile=tile, r_signed=r_signed, C=C)
        for s in range(n - 2):
            mu, sig = spread(q[s], sigma_est)
            out["mu"].append(mu)
            out["sigma"].append(sig)
            flag = 0 if (sig > 0 and np.isfinite(sig)) else FLAG_SIGMA_ZERO
            out["flags"].append(flag)
            if flag:
                continue
            for c in components(q[s], mu, sig, tau):
                c.update(branch=IMAGE, triple=s)
                out["cands"].append(c)
    out["q"] = q if keep_maps else None
    out["cube"] = None
    out["eta"] = None
    out["eta_mu"] = out["eta_sigma"] = None
    if (branches & FREQ) and n - 2 >= 4:
        cube = index_maps(X, mode=TILES, tile=tile, r_signed=r_signed, C=C)
        e = eta(cube, harm)
        mu, sig = spread(e, sigma_est)
        out["cube"], out["eta"], out["eta_mu"], out["eta_sigma"] = cube, e, mu, sig
        if sig > 0 and np.isfinite(sig):
            for c in components(e, mu, sig, tau):
                c.update(branch=FREQ, triple=-1)
                out["cands"].append(c)
    # per-pixel form: the spectrum of every cell's series of sliding q, for
    # every series length the tile branch accepts (n' >= 4)
    out["eta_px"] = None
    out["eta_px_mu"] = out["eta_px_sigma"] = None
    if (branches & FREQ_PIXEL) and mode == SLIDING and n - 2 >= 4:
        qp = q if q is not None else index_maps(X, mode=SLIDING, window=window, tile=tile, r_signed=r_signed, C=C)
        e = eta(qp, harm)
        mu, sig = spread(e, sigma_est)
        out["eta_px"], out["eta_px_mu"], out["eta_px_sigma"] = e, mu, sig
        if sig > 0 and np.isfinite(sig):
            for c in components(e, mu, sig, tau):
                c.update(branch=FREQ_PIXEL, triple=-1)
                out["cands"].append(c)
    return out


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops from now on; returns the count in effect."""
    L = lib()
    L.ref_set_threads(int(n))
    return int(L.ref_max_threads())
