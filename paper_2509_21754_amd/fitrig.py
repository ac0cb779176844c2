"""Python binding of the FITrig C ABI (``include/fitrig.h``).

Argument marshalling only: every step of the path runs in the HIP library
``libfitrig.so``. The functions named like the C entry points are thin
wrappers; :class:`Context` adds the torch-tensor convenience layer (device
memory and streams come from PyTorch, nothing else does).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

ABI_VERSION = 4

OK, E_INVAL, E_NOMEM, E_HIP, E_TRUNC, E_BUSY, E_NOTREADY, E_SCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
NOALLOC_SCRATCH_BYTES = 256 << 20
F32, F16, BF16 = 0, 1, 2
SLIDING, TILES = 0, 1
IMAGE, FREQ, FREQ_PIXEL = 1, 2, 4
MEAN_STD, MEDIAN_MAD = 0, 1
MAP_QTILDE, MAP_TLISI = 0, 1
FLAG_SIGMA_ZERO, FLAG_TRUNC = 1, 2

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfitrig.so")


class fitrig_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("window", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("branches", ctypes.c_int32),
        ("sigma_est", ctypes.c_int32),
        ("harm", ctypes.c_int32),
        ("r_signed", ctypes.c_int32),
        ("map_kind", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("C", ctypes.c_double),
        ("max_pixels", ctypes.c_int64),
        ("max_snap", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("max_segments", ctypes.c_int64),
    ]


class fitrig_candidate(ctypes.Structure):
    _fields_ = [
        ("branch", ctypes.c_int32),
        ("triple", ctypes.c_int32),
        ("label", ctypes.c_int64),
        ("n_pix", ctypes.c_int32),
        ("peak_y", ctypes.c_int32),
        ("peak_x", ctypes.c_int32),
        ("peak_z", ctypes.c_float),
        ("peak_q", ctypes.c_float),
        ("pad0", ctypes.c_int32),
        ("cy", ctypes.c_double),
        ("cx", ctypes.c_double),
        ("y0", ctypes.c_int32),
        ("x0", ctypes.c_int32),
        ("y1", ctypes.c_int32),
        ("x1", ctypes.c_int32),
    ]


class fitrig_stats(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_double),
        ("n_triples", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("mu", ctypes.POINTER(ctypes.c_double)),
        ("sigma", ctypes.POINTER(ctypes.c_double)),
        ("flags", ctypes.POINTER(ctypes.c_uint32)),
        ("eta_mu", ctypes.c_double),
        ("eta_sigma", ctypes.c_double),
        ("n_image_cand", ctypes.c_int64),
        ("n_freq_cand", ctypes.c_int64),
        ("n_freq_px_cand", ctypes.c_int64),
        ("eta_px_mu", ctypes.c_double),
        ("eta_px_sigma", ctypes.c_double),
        ("ran", ctypes.c_uint32),
        ("eta_flags", ctypes.c_uint32),
    ]


class fitrig_server_config(ctypes.Structure):
    _fields_ = [
        ("base", fitrig_config),
        ("n_slots", ctypes.c_int32),
        ("max_fields", ctypes.c_int32),
        ("mem_budget", ctypes.c_int64),
        ("cand_cap", ctypes.c_int64),
        ("freq_window", ctypes.c_int32),
        ("graphs", ctypes.c_int32),
    ]


class fitrig_result(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_int64),
        ("field_id", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("n_triples", ctypes.c_int32),
        ("first_triple", ctypes.c_int64),
        ("n_cand", ctypes.c_int64),
        ("cand", ctypes.POINTER(fitrig_candidate)),
        ("M", ctypes.c_double),
        ("t_submit_ns", ctypes.c_int64),
        ("t_start_ns", ctypes.c_int64),
        ("t_done_ns", ctypes.c_int64),
        ("freq_triples", ctypes.c_int32),
        ("replayed", ctypes.c_int32),
    ]


EXPORTS = (
    "fitrig_config_default",
    "fitrig_create",
    "fitrig_detect",
    "fitrig_detect_noalloc",
    "fitrig_detect_host",
    "fitrig_destroy",
    "fitrig_status_string",
    "fitrig_last_hip_error",
    "fitrig_abi_version",
    "fitrig_phase_times",
    "fitrig_server_config_default",
    "fitrig_server_create",
    "fitrig_submit",
    "fitrig_poll",
    "fitrig_release",
    "fitrig_server_destroy",
    "fitrig_interp_peaks",
    "fitrig_accumulate",
    "fitrig_accum_factor",
    "fitrig_index_prefix",
)
N_PHASES = 5
PHASES = ("index_pass", "spread", "image_select", "freq_branch", "host_copy")

_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """dlopen the HIP library; raises when it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"FITrig HIP library not built: {path} (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.fitrig_config_default.argtypes = [ctypes.POINTER(fitrig_config)]
    L.fitrig_config_default.restype = None
    L.fitrig_create.argtypes = [ctypes.POINTER(fitrig_config), ctypes.POINTER(vp)]
    L.fitrig_create.restype = i32
    L.fitrig_detect.argtypes = [vp, vp, i32, i32, i32, i32, dbl, ctypes.POINTER(fitrig_candidate), i64,
                                ctypes.POINTER(i64), vp, vp, vp, ctypes.POINTER(fitrig_stats), vp]
    L.fitrig_detect.restype = i32
    L.fitrig_detect_noalloc.argtypes = L.fitrig_detect.argtypes
    L.fitrig_detect_noalloc.restype = i32
    L.fitrig_detect_host.argtypes = [vp, vp, i32, i32, i32, i32, dbl, i32, ctypes.POINTER(fitrig_candidate), i64,
                                     ctypes.POINTER(i64), vp, ctypes.POINTER(fitrig_stats)]
    L.fitrig_detect_host.restype = i32
    L.fitrig_destroy.argtypes = [vp]
    L.fitrig_destroy.restype = i32
    L.fitrig_status_string.argtypes = [i32]
    L.fitrig_status_string.restype = ctypes.c_char_p
    L.fitrig_last_hip_error.argtypes = [vp]
    L.fitrig_last_hip_error.restype = i32
    L.fitrig_abi_version.argtypes = []
    L.fitrig_abi_version.restype = i32
    L.fitrig_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32]
    L.fitrig_phase_times.restype = i32
    L.fitrig_server_config_default.argtypes = [ctypes.POINTER(fitrig_server_config)]
    L.fitrig_server_config_default.restype = None
    L.fitrig_server_create.argtypes = [ctypes.POINTER(fitrig_server_config), ctypes.POINTER(vp)]
    L.fitrig_server_create.restype = i32
    L.fitrig_submit.argtypes = [vp, i64, vp, i32, i32, i32, i32, dbl, i32, ctypes.POINTER(i64)]
    L.fitrig_submit.restype = i32
    L.fitrig_poll.argtypes = [vp, i64, i32, ctypes.POINTER(fitrig_result)]
    L.fitrig_poll.restype = i32
    L.fitrig_release.argtypes = [vp, i64]
    L.fitrig_release.restype = i32
    L.fitrig_server_destroy.argtypes = [vp]
    L.fitrig_server_destroy.restype = i32
    L.fitrig_interp_peaks.argtypes = [vp, i32, i32, vp, vp, i32, i32, i32, vp, vp]
    L.fitrig_interp_peaks.restype = i32
    L.fitrig_accumulate.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]
    L.fitrig_accumulate.restype = i32
    L.fitrig_accum_factor.argtypes = [vp, i32, i32, i32, i32, dbl, i32, ctypes.POINTER(i32),
                                      ctypes.POINTER(ctypes.c_double), vp]
    L.fitrig_accum_factor.restype = i32
    L.fitrig_index_prefix.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, dbl, vp, vp]
    L.fitrig_index_prefix.restype = i32
    _lib = L
    return L


# ---- thin wrappers with the C names -----------------------------------------

def fitrig_config_default(**overrides) -> fitrig_config:
    cfg = fitrig_config()
    load().fitrig_config_default(ctypes.byref(cfg))
    for k, v in overrides.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def fitrig_create(cfg: fitrig_config) -> tuple[int, Optional[int]]:
    h = ctypes.c_void_p()
    rc = load().fitrig_create(ctypes.byref(cfg), ctypes.byref(h))
    return rc, (h.value if rc == OK else None)


def fitrig_detect(ctx, stack_ptr, dtype, n_snap, H, W, sigma, cand, cand_cap, n_cand, index_map, eta_map,
                  eta_px_map, stats, hip_stream) -> int:
    return load().fitrig_detect(ctx, stack_ptr, dtype, n_snap, H, W, sigma, cand, cand_cap, n_cand, index_map,
                                eta_map, eta_px_map, stats, hip_stream)


def fitrig_detect_noalloc(ctx, stack_ptr, dtype, n_snap, H, W, sigma, cand, cand_cap, n_cand, index_map, eta_map,
                          eta_px_map, stats, hip_stream) -> int:
    return load().fitrig_detect_noalloc(ctx, stack_ptr, dtype, n_snap, H, W, sigma, cand, cand_cap, n_cand,
                                        index_map, eta_map, eta_px_map, stats, hip_stream)


def fitrig_detect_host(ctx, host_ptr, dtype, n_snap, H, W, sigma, chunk_frames, cand, cand_cap, n_cand, eta_map,
                       stats) -> int:
    return load().fitrig_detect_host(ctx, host_ptr, dtype, n_snap, H, W, sigma, chunk_frames, cand, cand_cap, n_cand,
                                     eta_map, stats)


def fitrig_destroy(ctx) -> int:
    return load().fitrig_destroy(ctx)


def fitrig_status_string(code: int) -> str:
    return load().fitrig_status_string(code).decode()


def fitrig_last_hip_error(ctx) -> int:
    return load().fitrig_last_hip_error(ctx)


def fitrig_abi_version() -> int:
    return load().fitrig_abi_version()


def fitrig_phase_times(ctx) -> list:
    buf = (ctypes.c_double * N_PHASES)()
    n = load().fitrig_phase_times(ctx, buf, N_PHASES)
    return list(buf[:max(n, 0)])


def fitrig_server_config_default(**overrides) -> fitrig_server_config:
    cfg = fitrig_server_config()
    load().fitrig_server_config_default(ctypes.byref(cfg))
    for k, v in overrides.items():
        if hasattr(cfg, k):
            setattr(cfg, k, v)
        elif hasattr(cfg.base, k):
            setattr(cfg.base, k, v)
        else:
            raise KeyError(k)
    return cfg


def fitrig_server_create(cfg: fitrig_server_config) -> tuple[int, Optional[int]]:
    h = ctypes.c_void_p()
    rc = load().fitrig_server_create(ctypes.byref(cfg), ctypes.byref(h))
    return rc, (h.value if rc == OK else None)


def fitrig_submit(srv, field_id, stack_ptr, dtype, n_snap, H, W, sigma, blocking, ticket) -> int:
    return load().fitrig_submit(srv, field_id, stack_ptr, dtype, n_snap, H, W, sigma, blocking, ticket)


def fitrig_poll(srv, ticket, wait, out) -> int:
    return load().fitrig_poll(srv, ticket, wait, out)


def fitrig_release(srv, ticket) -> int:
    return load().fitrig_release(srv, ticket)


def fitrig_server_destroy(srv) -> int:
    return load().fitrig_server_destroy(srv)


INTERP_BILINEAR, INTERP_BICUBIC, INTERP_SPLINE, INTERP_MAKIMA = 0, 1, 2, 3


def fitrig_interp_peaks(map_ptr, H: int, W: int, py, px, n: int, method: int, sub: int, out, stream) -> int:
    return load().fitrig_interp_peaks(map_ptr, H, W, py, px, n, method, sub, out, stream)


def interp_peaks(value_map, peaks, method: int = INTERP_SPLINE, sub: int = 16, stream=None):
    """Sub-cell positions of peak cells of a 2-D FP32 device map.

    peaks: sequence of (y, x) cells. Returns a float64 array [n, 3] of
    (y, x, interpolated value)."""
    import numpy as np

    if not value_map.is_cuda or value_map.dim() != 2 or not value_map.is_contiguous():
        raise ValueError("value_map must be a contiguous 2-D device tensor")
    if str(value_map.dtype) != "torch.float32":
        raise ValueError("value_map must be float32")
    pk = np.ascontiguousarray(np.asarray(peaks, dtype=np.int32).reshape(-1, 2))
    n = pk.shape[0]
    py = np.ascontiguousarray(pk[:, 0])
    px = np.ascontiguousarray(pk[:, 1])
    out = np.zeros((n, 3), dtype=np.float64)
    H, W = value_map.shape
    st = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
    rc = fitrig_interp_peaks(ctypes.c_void_p(value_map.data_ptr()), H, W, py.ctypes.data_as(ctypes.c_void_p),
                             px.ctypes.data_as(ctypes.c_void_p), n, int(method), int(sub),
                             out.ctypes.data_as(ctypes.c_void_p), st)
    if rc != OK:
        raise FitrigError(rc, "fitrig_interp_peaks")
    return out


# ---- torch convenience layer --------------------------------------------------

class FitrigError(RuntimeError):
    def __init__(self, code: int, where: str, hip: int = 0):
        super().__init__(f"{where}: {fitrig_status_string(code)} ({code}), hip error {hip}")
        self.code = code


def _dtype_code(t) -> int:
    import torch

    return {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}[t.dtype]


_CAND_KEYS = ("branch", "triple", "label", "n_pix", "peak_y", "peak_x", "peak_z", "peak_q", "cy", "cx",
              "y0", "x0", "y1", "x1")


_CAND_NP = None


def cand_dtype():
    """numpy structured dtype of fitrig_candidate (72 bytes, C layout)."""
    global _CAND_NP
    if _CAND_NP is None:
        import numpy as np

        _CAND_NP = np.ctypeslib.as_array((fitrig_candidate * 1)()).dtype
    return _CAND_NP


def _cand_array(addr: int, k: int):
    """Copy k records at host address addr into a new numpy array (a raw
    byte copy: numpy's field-wise copy of this dtype is ~10x slower)."""
    import numpy as np

    out = np.empty(k, dtype=cand_dtype())
    if k:
        ctypes.memmove(out.ctypes.data, addr, k * ctypes.sizeof(fitrig_candidate))
    return out


def _rec_dict(r) -> dict:
    d = {k: r[k].item() for k in _CAND_KEYS}
    # float fields come from float32 storage
    d["peak_z"] = float(r["peak_z"])
    d["peak_q"] = float(r["peak_q"])
    return d


class Context:
    """Owns a fitrig_ctx; ``detect`` takes device tensors."""

    def __init__(self, **cfg):
        self.cfg = fitrig_config_default(**cfg)
        rc, h = fitrig_create(self.cfg)
        if rc != OK:
            raise FitrigError(rc, "fitrig_create")
        self.handle = h

    def phase_times(self) -> dict:
        """Per-phase milliseconds of the last detect (config profile=1)."""
        return dict(zip(PHASES, fitrig_phase_times(self.handle)))

    def close(self):
        if getattr(self, "handle", None):
            fitrig_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _buffers(self, cand_cap: int, np_: int):
        b = getattr(self, "_buf", None)
        if b is None or b["cap"] < cand_cap or b["np"] < np_:
            cap, npb = max(cand_cap, 1), max(np_, 1)
            b = {"cap": cap, "np": npb, "cand": (fitrig_candidate * cap)(),
                 "mu": (ctypes.c_double * npb)(), "sg": (ctypes.c_double * npb)(),
                 "fl": (ctypes.c_uint32 * npb)(), "n": ctypes.c_int64(), "st": fitrig_stats()}
            b["st"].mu = ctypes.cast(b["mu"], ctypes.POINTER(ctypes.c_double))
            b["st"].sigma = ctypes.cast(b["sg"], ctypes.POINTER(ctypes.c_double))
            b["st"].flags = ctypes.cast(b["fl"], ctypes.POINTER(ctypes.c_uint32))
            self._buf = b
        return b

    def detect(self, stack, sigma: float, *, cand_cap: int = 1 << 16, index_map=None, eta_map=None,
               eta_px_map=None, stream=None, raise_on_trunc: bool = False, as_dicts: bool = True):
        """Run the path on ``stack`` ([n][H][W] device tensor, f32/f16/bf16).

        Synchronous: the library runs on torch's current stream (or ``stream``)
        as an asynchronous call and this method synchronises that stream
        before reading the results. Returns (candidates, stats (dict),
        status). Candidates are a list of dicts, or with ``as_dicts=False`` a
        numpy structured array over page-locked memory of its own, which the
        device writes the records into directly (no host copy)."""
        import numpy as np
        import torch

        if not stack.is_cuda or not stack.is_contiguous() or stack.dim() != 3:
            raise ValueError("stack must be a contiguous 3-D device tensor")
        n, H, W = stack.shape
        np_ = max(n - 2, 0)
        b = self._buffers(cand_cap, np_)
        for m in (index_map, eta_map, eta_px_map):
            if m is not None and (not m.is_cuda or m.dtype != torch.float32 or not m.is_contiguous()):
                raise ValueError("maps must be contiguous float32 device tensors")
        if stream is None:
            stream = torch.cuda.current_stream(stack.device)
        # a null stream handle (the legacy default stream) makes the call
        # synchronous on the context's stream; any other stream makes it
        # asynchronous on that stream
        # the records go to page-locked memory (torch's cached host blocks):
        # the library writes mapped page-locked arrays from the device. The
        # first call of a size leaves four such blocks in torch's cache, so
        # later calls take cached blocks (a fresh page-locked allocation costs
        # milliseconds) while the caller keeps a few earlier results alive.
        nbytes = max(cand_cap, 1) * ctypes.sizeof(fitrig_candidate)
        if getattr(self, "_pinned_warm", 0) < nbytes:
            warm = [torch.empty(nbytes, dtype=torch.uint8, pin_memory=True) for _ in range(4)]
            del warm
            self._pinned_warm = nbytes
        ct = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        cand = ctypes.cast(ctypes.c_void_p(ct.data_ptr()), ctypes.POINTER(fitrig_candidate))
        rc = self.enqueue(stack, sigma, b, cand_cap, index_map, eta_map, eta_px_map, stream, cand=cand)
        if rc not in (OK, E_TRUNC):
            raise FitrigError(rc, "fitrig_detect", fitrig_last_hip_error(self.handle))
        stream.synchronize()
        rc = b["st"].status
        if rc == E_TRUNC and raise_on_trunc:
            raise FitrigError(rc, "fitrig_detect")
        return self._results(b, cand_cap, np_, rc, as_dicts, cand_t=ct)

    def _results(self, b, cand_cap, np_, rc, as_dicts, cand_t=None):
        ncand = b["n"].value
        k = min(ncand, cand_cap)
        if cand_t is not None:
            # a view of the page-locked records (it keeps the block alive)
            arr = cand_t.numpy()[: k * ctypes.sizeof(fitrig_candidate)].view(cand_dtype())
        else:
            arr = _cand_array(ctypes.addressof(b["cand"]), k)
        cands = [_rec_dict(r) for r in arr] if as_dicts else arr
        st = b["st"]
        stats = dict(M=st.M, n_triples=st.n_triples, mu=list(b["mu"][:np_]), sigma=list(b["sg"][:np_]),
                     flags=list(b["fl"][:np_]), eta_mu=st.eta_mu, eta_sigma=st.eta_sigma,
                     eta_px_mu=st.eta_px_mu, eta_px_sigma=st.eta_px_sigma, ran=st.ran, eta_flags=st.eta_flags,
                     n_image_cand=st.n_image_cand, n_freq_cand=st.n_freq_cand,
                     n_freq_px_cand=st.n_freq_px_cand, n_cand=ncand, status=st.status)
        return cands, stats, rc

    def detect_host(self, stack, sigma: float, chunk_frames: int, *, cand_cap: int = 1 << 16, eta_map=None,
                    as_dicts: bool = True):
        """Run the path on a stack in host memory ([n][H][W] CPU tensor,
        f32/f16/bf16; pinned memory is copied directly, pageable memory through
        page-locked staging buffers filled by host threads), streamed in chunks
        of ``chunk_frames`` frames. Returns (candidates, stats, status) as
        ``detect``."""
        import torch

        if stack.is_cuda or not stack.is_contiguous() or stack.dim() != 3:
            raise ValueError("stack must be a contiguous 3-D host tensor")
        if eta_map is not None and (not eta_map.is_cuda or eta_map.dtype != torch.float32 or
                                    not eta_map.is_contiguous()):
            raise ValueError("eta_map must be a contiguous float32 device tensor")
        n, H, W = stack.shape
        np_ = max(n - 2, 0)
        b = self._buffers(cand_cap, np_)
        rc = fitrig_detect_host(self.handle, ctypes.c_void_p(stack.data_ptr()), _dtype_code(stack), n, H, W,
                                float(sigma), int(chunk_frames), b["cand"], cand_cap, ctypes.byref(b["n"]),
                                ctypes.c_void_p(eta_map.data_ptr()) if eta_map is not None else None,
                                ctypes.byref(b["st"]))
        if rc not in (OK, E_TRUNC):
            raise FitrigError(rc, "fitrig_detect_host", fitrig_last_hip_error(self.handle))
        return self._results(b, cand_cap, np_, rc, as_dicts)

    def enqueue(self, stack, sigma, b, cand_cap, index_map, eta_map, eta_px_map, stream, cand=None) -> int:
        """The asynchronous C call on ``stream`` with the host buffers ``b``
        (from ``_buffers``) and the candidate array ``cand`` (default
        ``b["cand"]``), which must stay alive until the stream has run it."""
        n, H, W = stack.shape
        ptr = lambda m: ctypes.c_void_p(m.data_ptr()) if m is not None else None  # noqa: E731
        return fitrig_detect(self.handle, ctypes.c_void_p(stack.data_ptr()), _dtype_code(stack), n, H, W,
                             float(sigma), b["cand"] if cand is None else cand, cand_cap, ctypes.byref(b["n"]),
                             ptr(index_map), ptr(eta_map), ptr(eta_px_map), ctypes.byref(b["st"]),
                             ctypes.c_void_p(stream.cuda_stream))


class Server:
    """Owns a fitrig_server; stacks are device tensors that must stay alive
    (and unchanged) until their ticket is done."""

    def __init__(self, n_slots: int = 4, max_fields: int = 64, mem_budget: int = 0, cand_cap: int = 1 << 16,
                 freq_window: int = 0, graphs: int = 1, **base):
        self.cfg = fitrig_server_config_default(n_slots=n_slots, max_fields=max_fields, mem_budget=mem_budget,
                                                cand_cap=cand_cap, freq_window=freq_window, graphs=graphs,
                                                **base)
        rc, h = fitrig_server_create(self.cfg)
        if rc != OK:
            raise FitrigError(rc, "fitrig_server_create")
        self.handle = h
        self._keep = {}

    def submit(self, field_id: int, stack, sigma: float, blocking: bool = True):
        """Ticket, or None when a non-blocking submit is not admitted."""
        if not stack.is_cuda or not stack.is_contiguous() or stack.dim() != 3:
            raise ValueError("stack must be a contiguous 3-D device tensor")
        n, H, W = stack.shape
        t = ctypes.c_int64()
        rc = fitrig_submit(self.handle, int(field_id), ctypes.c_void_p(stack.data_ptr()), _dtype_code(stack), n, H,
                           W, float(sigma), 1 if blocking else 0, ctypes.byref(t))
        if rc == E_BUSY and not blocking:
            return None
        if rc != OK:
            raise FitrigError(rc, "fitrig_submit")
        self._keep[t.value] = stack
        return t.value

    def poll(self, ticket: int, wait: bool = True, as_dicts: bool = True):
        """Result dict (candidates, timing), or None if not ready (wait=False)."""
        import numpy as np

        r = fitrig_result()
        rc = fitrig_poll(self.handle, ticket, 1 if wait else 0, ctypes.byref(r))
        if rc == E_NOTREADY:
            return None
        if rc != OK:
            raise FitrigError(rc, "fitrig_poll")
        k = min(r.n_cand, self.cfg.cand_cap)
        arr = _cand_array(ctypes.cast(r.cand, ctypes.c_void_p).value, k) if (k and r.cand) else _cand_array(0, 0)
        return dict(ticket=r.ticket, field_id=r.field_id, status=r.status, n_triples=r.n_triples,
                    first_triple=r.first_triple, n_cand=r.n_cand, M=r.M, freq_triples=r.freq_triples,
                    replayed=r.replayed,
                    cands=[_rec_dict(x) for x in arr] if as_dicts else arr,
                    t_submit_ns=r.t_submit_ns, t_start_ns=r.t_start_ns, t_done_ns=r.t_done_ns)

    def release(self, ticket: int):
        rc = fitrig_release(self.handle, ticket)
        if rc != OK:
            raise FitrigError(rc, "fitrig_release")
        self._keep.pop(ticket, None)

    def close(self):
        if getattr(self, "handle", None):
            fitrig_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---- snapshot accumulation ----------------------------------------------------

def fitrig_accumulate(stack_ptr, dtype, n_snap, H, W, K, out_ptr, hip_stream) -> int:
    return load().fitrig_accumulate(stack_ptr, dtype, n_snap, H, W, K, out_ptr, hip_stream)


def fitrig_accum_factor(stack_ptr, dtype, n_snap, H, W, gamma, k_max, K_out, contrast, hip_stream) -> int:
    return load().fitrig_accum_factor(stack_ptr, dtype, n_snap, H, W, gamma, k_max, K_out, contrast, hip_stream)


def accumulate(stack, K: int):
    """Sums of K consecutive snapshots ([n // K][H][W] float32 device tensor),
    enqueued on torch's current stream."""
    import torch

    if not stack.is_cuda or not stack.is_contiguous() or stack.dim() != 3:
        raise ValueError("stack must be a contiguous 3-D device tensor")
    n, H, W = stack.shape
    out = torch.empty((max(n // max(K, 1), 0), H, W), dtype=torch.float32, device=stack.device)
    rc = fitrig_accumulate(ctypes.c_void_p(stack.data_ptr()), _dtype_code(stack), n, H, W, int(K),
                           ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != OK:
        raise FitrigError(rc, "fitrig_accumulate")
    return out


def accum_factor(stack, gamma: float, k_max: int):
    """(K, [C(1) .. C(k_max)]): the automatic accumulation factor, on torch's current stream."""
    import torch

    if not stack.is_cuda or not stack.is_contiguous() or stack.dim() != 3:
        raise ValueError("stack must be a contiguous 3-D device tensor")
    n, H, W = stack.shape
    K = ctypes.c_int32()
    C = (ctypes.c_double * max(int(k_max), 1))()
    rc = fitrig_accum_factor(ctypes.c_void_p(stack.data_ptr()), _dtype_code(stack), n, H, W, float(gamma),
                             int(k_max), ctypes.byref(K), C, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != OK:
        raise FitrigError(rc, "fitrig_accum_factor")
    return K.value, list(C)[:k_max]


# ---- window sums from prefix sums (comparison variant) -----------------------

def fitrig_index_prefix(stack_ptr, dtype, n_snap, H, W, window, prefix_bits, r_signed, C, map_ptr, hip_stream) -> int:
    return load().fitrig_index_prefix(stack_ptr, dtype, n_snap, H, W, window, prefix_bits, r_signed, C, map_ptr,
                                      hip_stream)


def index_prefix(stack, window: int, prefix_bits: int = 64, r_signed: int = 0, C: float = 1e-6, out=None):
    """q maps of every triple ([n-2][H][W] float32 device tensor) with the window
    sums read from integral images in FP64 (or FP32), on torch's current stream."""
    import torch

    if not stack.is_cuda or not stack.is_contiguous() or stack.dim() != 3:
        raise ValueError("stack must be a contiguous 3-D device tensor")
    n, H, W = stack.shape
    if out is None:
        out = torch.empty((max(n - 2, 0), H, W), dtype=torch.float32, device=stack.device)
    rc = fitrig_index_prefix(ctypes.c_void_p(stack.data_ptr()), _dtype_code(stack), n, H, W, int(window),
                             int(prefix_bits), int(r_signed), float(C), ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != OK:
        raise FitrigError(rc, "fitrig_index_prefix")
    return out
