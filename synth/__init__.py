"""Seeded synthetic snapshot stacks (input generator shared by tests, smoke
check and benchmark; it holds none of the detection arithmetic).

The paper evaluates on simulated MeerKAT / SKA AA2 dirty snapshots and on a
real MeerKAT measurement set (Sec. 3); none of those data exist here. These
stacks stand in for them with the shapes and content the workloads name:

* noise: independent N(0, 1) per pixel per frame, added after convolution;
* PSF: a K x K stamp, K = min(257, largest odd <= H/2): a Gaussian core of
  3 px FWHM plus sidelobes taken from the real part of the inverse FFT of a
  seeded random 5 % uv-sampling mask (fft-shifted, divided by its centre
  value, centre set to 0); core + sidelobes, normalised to peak 1;
* steady sources: integer positions uniform over the image, stamps clipped
  at the edge, constant amplitude over frames;
* pulsars: either a full-amplitude boxcar in every 8th frame (frames with
  k % 8 == 7, 0-based), or a periodic truncated-Gaussian pulse (10 % duty,
  sigma = duty / 4, truncated at +-2 sigma) integrated over each frame
  (Sec. 3.1 describes this profile).

Everything is drawn from numpy's PCG64 seeded per stack; frame noise comes
from a torch generator on the target device seeded per (stack, frame), so a
stack is reproducible on a given device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Sequence

import numpy as np

FWHM_PX = 3.0
UV_FILL = 0.05


@dataclass(frozen=True)
class StackSpec:
    name: str
    H: int
    W: int
    n: int
    dtype: str = "f32"            # storage dtype: f32 | f16 | bf16
    window: int = 7
    taus: Sequence[float] = (6.0,)
    n_steady: int = 0
    steady_amp: Optional[float] = None        # fixed amplitude, else log-uniform
    steady_range: tuple = (5.0, 100.0)
    n_pulsar: int = 0
    pulsar_kind: str = "every8"               # every8 | periodic
    pulsar_amp: Optional[float] = None        # fixed; None: see pulsar_rel / range
    pulsar_rel: Optional[float] = None        # amplitude = nearest steady * rel
    pulsar_range: tuple = (0.5, 3.0)
    period_range: tuple = (4, 16)
    seed: int = 0


# The five workloads (seeds 1000 + index).
WORKLOADS = {
    "c0": StackSpec("c0", 256, 256, 32, "f32", 7, (6.0,), n_steady=5, steady_amp=20.0,
                    n_pulsar=1, pulsar_kind="every8", pulsar_amp=1.0, seed=1000),
    "c1": StackSpec("c1", 4096, 4096, 64, "f32", 7, (5.0, 6.0, 7.0), n_steady=200,
                    n_pulsar=10, pulsar_kind="periodic", seed=1001),
    "c2": StackSpec("c2", 16384, 16384, 32, "f32", 9, (6.0,), n_steady=2000,
                    n_pulsar=50, pulsar_kind="every8", pulsar_rel=1.0 / 20.0, seed=1002),
    "c3": StackSpec("c3", 50000, 50000, 16, "f16", 9, (6.0,), n_steady=18626,
                    n_pulsar=466, pulsar_kind="every8", pulsar_rel=1.0 / 20.0, seed=1003),
}


def scaled(spec: StackSpec, H: int, W: int, n: Optional[int] = None,
           seed: Optional[int] = None, dtype: Optional[str] = None) -> StackSpec:
    """The same recipe at another size, source counts scaled by area."""
    area = (H * W) / float(spec.H * spec.W)
    ns = int(round(spec.n_steady * area)) if spec.n_steady else 0
    npul = int(round(spec.n_pulsar * area)) if spec.n_pulsar else 0
    if spec.n_steady and ns == 0:
        ns = 1
    if spec.n_pulsar and npul == 0:
        npul = 1
    return replace(spec, H=H, W=W, n=spec.n if n is None else n,
                   n_steady=ns, n_pulsar=npul,
                   seed=spec.seed if seed is None else seed,
                   dtype=spec.dtype if dtype is None else dtype)


def psf_size(H: int, W: int) -> int:
    k = min(257, min(H, W) // 2)
    if k % 2 == 0:
        k -= 1
    return max(k, 1)


def gaussian_core(K: int, fwhm: float = FWHM_PX) -> np.ndarray:
    sig = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    c = K // 2
    yy, xx = np.mgrid[0:K, 0:K]
    return np.exp(-((yy - c) ** 2 + (xx - c) ** 2) / (2.0 * sig * sig))


def make_psf(K: int, rng: np.random.Generator) -> np.ndarray:
    core = gaussian_core(K)
    if K < 3:
        return core / core.max()
    mask = (rng.random((K, K)) < UV_FILL).astype(np.float64)
    side = np.real(np.fft.fftshift(np.fft.ifft2(mask)))
    c = K // 2
    if side[c, c] != 0:
        side = side / side[c, c]
    side[c, c] = 0.0
    p = core + side
    return p / p.max()


def _add_stamp(img, psf, y: int, x: int, amp: float):
    """img[y + dy, x + dx] += amp * psf[c + dy, c + dx], clipped at the edge."""
    H, W = img.shape
    K = psf.shape[0]
    c = K // 2
    y0, y1 = max(0, y - c), min(H, y - c + K)
    x0, x1 = max(0, x - c), min(W, x - c + K)
    if y0 >= y1 or x0 >= x1:
        return
    img[y0:y1, x0:x1] += amp * psf[y0 - (y - c):y1 - (y - c), x0 - (x - c):x1 - (x - c)]


def _phi(z: float) -> float:
    return 0.5 * (1.0 + math.erf(z / math.sqrt(2.0)))


def pulse_frame_weights(n: int, period: float, phase: float, duty: float = 0.1) -> np.ndarray:
    """Fraction of a truncated-Gaussian pulse (width duty*period, sigma =
    width/4, truncated at +-2 sigma) that falls into each frame [k, k+1),
    normalised so that a pulse wholly inside one frame gives weight 1."""
    width = duty * period
    sig = width / 4.0
    norm = _phi(2.0) - _phi(-2.0)
    w = np.zeros(n)
    m = 0
    while True:
        tc = phase + m * period
        if tc - width / 2 > n:
            break
        lo_t, hi_t = tc - width / 2, tc + width / 2
        for k in range(max(0, int(math.floor(lo_t))), min(n, int(math.ceil(hi_t)) + 1)):
            a, b = max(k, lo_t), min(k + 1, hi_t)
            if b > a:
                w[k] += (_phi((b - tc) / sig) - _phi((a - tc) / sig)) / norm
        m += 1
    return w


@dataclass
class SkyModel:
    psf: np.ndarray
    steady_yx: np.ndarray
    steady_amp: np.ndarray
    pulsar_yx: np.ndarray
    pulsar_amp: np.ndarray
    pulsar_w: np.ndarray        # [n_pulsar][n] frame weights


def sky_model(spec: StackSpec) -> SkyModel:
    rng = np.random.default_rng(spec.seed)
    K = psf_size(spec.H, spec.W)
    psf = make_psf(K, rng)
    sy = rng.integers(0, spec.H, spec.n_steady)
    sx = rng.integers(0, spec.W, spec.n_steady)
    if spec.steady_amp is not None:
        sa = np.full(spec.n_steady, float(spec.steady_amp))
    else:
        lo, hi = spec.steady_range
        sa = np.exp(rng.uniform(math.log(lo), math.log(hi), spec.n_steady))
    py = rng.integers(0, spec.H, spec.n_pulsar)
    px = rng.integers(0, spec.W, spec.n_pulsar)
    if spec.pulsar_amp is not None:
        pa = np.full(spec.n_pulsar, float(spec.pulsar_amp))
    elif spec.pulsar_rel is not None:
        pa = np.empty(spec.n_pulsar)
        for i in range(spec.n_pulsar):
            if spec.n_steady:
                d2 = (sy - py[i]) ** 2 + (sx - px[i]) ** 2
                pa[i] = sa[int(np.argmin(d2))] * spec.pulsar_rel
            else:
                pa[i] = spec.pulsar_rel
    else:
        pa = rng.uniform(spec.pulsar_range[0], spec.pulsar_range[1], spec.n_pulsar)
    pw = np.zeros((spec.n_pulsar, spec.n))
    for i in range(spec.n_pulsar):
        if spec.pulsar_kind == "every8":
            pw[i, 7::8] = 1.0
        else:
            P = int(rng.integers(spec.period_range[0], spec.period_range[1] + 1))
            ph = float(rng.uniform(0.0, P))
            pw[i] = pulse_frame_weights(spec.n, P, ph)
    return SkyModel(psf, np.stack([sy, sx], 1), sa, np.stack([py, px], 1), pa, pw)


_TORCH_DT = {"f32": "float32", "f16": "float16", "bf16": "bfloat16"}


def make_stack(spec: StackSpec, device="cpu", noise_sigma: float = 1.0, on_frame=None):
    """Materialise the stack [n][H][W] in the storage dtype on ``device``.

    ``on_frame(k, frame)``, if given, sees each float32 frame before it is
    rounded to the storage dtype (for crops of the unquantised values)."""
    import torch

    sky = sky_model(spec)
    dev = torch.device(device)
    psf = torch.tensor(sky.psf, dtype=torch.float32, device=dev)
    steady = torch.zeros((spec.H, spec.W), dtype=torch.float32, device=dev)
    for (y, x), a in zip(sky.steady_yx, sky.steady_amp):
        _add_stamp(steady, psf, int(y), int(x), float(a))
    # pulsar images: group pulsars that share identical frame weights
    groups: dict = {}
    for i in range(len(sky.pulsar_amp)):
        key = tuple(np.round(sky.pulsar_w[i], 12))
        groups.setdefault(key, []).append(i)
    pimgs = []
    for key, idx in groups.items():
        img = torch.zeros((spec.H, spec.W), dtype=torch.float32, device=dev)
        for i in idx:
            _add_stamp(img, psf, int(sky.pulsar_yx[i, 0]), int(sky.pulsar_yx[i, 1]),
                       float(sky.pulsar_amp[i]))
        pimgs.append((np.array(key), img))
    out = torch.empty((spec.n, spec.H, spec.W), dtype=getattr(torch, _TORCH_DT[spec.dtype]),
                      device=dev)
    gen = torch.Generator(device=dev)
    frame = torch.empty((spec.H, spec.W), dtype=torch.float32, device=dev)
    for k in range(spec.n):
        gen.manual_seed(spec.seed * 1_000_003 + k)
        torch.randn((spec.H, spec.W), generator=gen, dtype=torch.float32, device=dev, out=frame)
        if noise_sigma != 1.0:
            frame.mul_(noise_sigma)
        frame.add_(steady)
        for w, img in pimgs:
            if w[k] != 0.0:
                frame.add_(img, alpha=float(w[k]))
        if on_frame is not None:
            on_frame(k, frame)
        out[k].copy_(frame)
    return out


def spec(name: str, **over) -> StackSpec:
    base = WORKLOADS[name]
    if "H" in over or "W" in over:
        s = scaled(base, over.pop("H", base.H), over.pop("W", base.W), over.pop("n", None),
                   over.pop("seed", None), over.pop("dtype", None))
        return replace(s, **over) if over else s
    return replace(base, **over) if over else base


def serving_requests(count: int, rate_hz: float = 40.0, seed: int = 1004,
                     sizes=(2048, 4096, 8192), lengths=(16, 32, 128), n_fields: int = 16):
    """Poisson arrivals for the serving workload: each request names a field
    (a fixed size class and storage dtype per field, fp16 / fp32 50 / 50) and a
    snapshot count."""
    rng = np.random.default_rng(seed)
    field_size = rng.choice(sizes, n_fields)
    field_dtype = np.where(rng.random(n_fields) < 0.5, "f16", "f32")
    t = np.cumsum(rng.exponential(1.0 / rate_hz, count))
    reqs = []
    for i in range(count):
        f = int(rng.integers(0, n_fields))
        reqs.append(dict(t=float(t[i]), field=f, size=int(field_size[f]),
                         n=int(rng.choice(lengths)), dtype=str(field_dtype[f])))
    return reqs
