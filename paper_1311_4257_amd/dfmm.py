"""Thin ctypes binding of libdfmm (the C ABI declared in include/dfmm.h).

Argument marshalling only: every step of the matvec runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  If the shared
library has not been built, importing this module raises ImportError -- there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfmm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libdfmm.so not built ({LIB_PATH}); run __graft_entry__.build()")

# torch first: the library's HIP runtime dependency must resolve to the runtime
# torch has loaded.  Loaded the other way round, the process holds two HIP
# runtimes and whichever initializes second finds no device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

STAGES = ["permute_in", "s2m", "hf_m2m", "hf_m2l", "hf_reduce", "hf_l2l", "lf_m2l", "lf_reduce",
          "leaf_eval", "zero", "near_field"]

OK, EINVAL, EDOMAIN, EUNSUPPORTED, ENOMEM, EDEVICE, EIO = 0, -1, -2, -3, -4, -5, -6  # dfmm_status
MAX_BATCH = 32  # DFMM_MAX_BATCH
NOALLOC_MAX_BYTES = 64 << 20  # DFMM_NOALLOC_MAX_BYTES
PREC_FP32, PREC_FP16X3, PREC_BF16X3, PREC_FP64 = 0, 1, 2, 3  # DFMM_PREC_*

EXPORT_PERM, EXPORT_BOXES, EXPORT_PAIRS, EXPORT_NEAR, EXPORT_OUT_SLOTS, EXPORT_IN_SLOTS = 1, 2, 3, 4, 5, 6
EXPORT_LEAVES = 7

ABI_FUNCTIONS = [
    "dfmm_status_string", "dfmm_last_error", "dfmm_opset_build", "dfmm_opset_create",
    "dfmm_opset_set", "dfmm_opset_get", "dfmm_opset_info", "dfmm_opset_save", "dfmm_opset_load",
    "dfmm_opset_destroy", "dfmm_options_default", "dfmm_plan", "dfmm_plan_ex", "dfmm_apply",
    "dfmm_apply_batch", "dfmm_workspace_bytes", "dfmm_apply_ws", "dfmm_apply_noalloc", "dfmm_destroy",
    "dfmm_plan_info", "dfmm_export",
    "dfmm_set_timing", "dfmm_stage_times",
    "dfmm_server_create", "dfmm_server_submit", "dfmm_server_wait", "dfmm_server_drain", "dfmm_server_now",
    "dfmm_server_passes", "dfmm_server_pass", "dfmm_server_footprint", "dfmm_server_destroy",
]


class Options(C.Structure):
    _fields_ = [("eps", C.c_double), ("opset", C.c_void_p), ("cache_dir", C.c_char_p),
                ("device", C.c_int), ("precision", C.c_int), ("leaf_width", C.c_double),
                ("tol_factor", C.c_double), ("hbm_budget_bytes", C.c_uint64), ("leaf_max", C.c_int),
                ("lf_levels", C.c_int), ("reserved", C.c_int * 2)]


class Info(C.Structure):
    _fields_ = [("N", C.c_int64), ("K", C.c_double), ("depth", C.c_int), ("w_top", C.c_int),
                ("nlevels_hf", C.c_int), ("boxes", C.c_int64 * 32), ("pairs", C.c_int64 * 32),
                ("offsets", C.c_int64 * 32), ("out_slots", C.c_int64 * 32),
                ("in_slots", C.c_int64 * 32), ("rank", C.c_int * 32), ("near_pairs", C.c_int64),
                ("near_point_pairs", C.c_int64), ("flops_m2l_hf", C.c_double),
                ("flops_m2l_lf", C.c_double), ("plan_seconds", C.c_double),
                ("device_bytes", C.c_int64), ("bytes_m2l_op", C.c_double),
                ("bytes_m2l_vec", C.c_double), ("flops_m2l_level", C.c_double * 32), ("tau", C.c_double),
                ("flops_m2m", C.c_double), ("flops_l2l", C.c_double),
                ("bytes_l2l_op", C.c_double), ("bytes_l2l_vec", C.c_double), ("leaves", C.c_int64),
                ("depth_max", C.c_int), ("reserved_i", C.c_int)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_sig = {
    "dfmm_status_string": (C.c_char_p, [C.c_int]),
    "dfmm_last_error": (C.c_char_p, []),
    "dfmm_opset_build": (C.c_int, [C.c_double, C.c_int, C.c_char_p, C.POINTER(_P)]),
    "dfmm_opset_create": (C.c_int, [C.c_double, C.c_int, C.POINTER(_P)]),
    "dfmm_opset_set": (C.c_int, [_P, C.c_double, C.c_int, C.c_int, _D, _D, _D]),
    "dfmm_opset_get": (C.c_int, [_P, C.c_double, C.c_int, C.POINTER(C.c_int), _D, _D, _D]),
    "dfmm_opset_info": (C.c_int, [_P, _D, C.POINTER(C.c_int)]),
    "dfmm_opset_save": (C.c_int, [_P, C.c_char_p]),
    "dfmm_opset_load": (C.c_int, [C.c_char_p, C.POINTER(_P)]),
    "dfmm_opset_destroy": (None, [_P]),
    "dfmm_options_default": (None, [C.POINTER(Options)]),
    "dfmm_plan": (C.c_int, [_D, C.c_int64, C.c_double, C.c_double, C.POINTER(_P)]),
    "dfmm_plan_ex": (C.c_int, [_D, C.c_int64, C.c_double, C.POINTER(Options), C.POINTER(_P)]),
    "dfmm_apply": (C.c_int, [_P, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "dfmm_apply_batch": (C.c_int, [_P, C.c_int, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_int), C.c_void_p]),
    "dfmm_workspace_bytes": (C.c_int, [_P, C.c_int, C.POINTER(C.c_size_t)]),
    "dfmm_apply_ws": (C.c_int, [_P, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dfmm_apply_noalloc": (C.c_int, [_P, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "dfmm_destroy": (None, [_P]),
    "dfmm_plan_info": (C.c_int, [_P, C.POINTER(Info)]),
    "dfmm_export": (C.c_int, [_P, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_size_t)]),
    "dfmm_set_timing": (C.c_int, [_P, C.c_int]),
    "dfmm_stage_times": (C.c_int, [_P, _D, C.POINTER(C.c_int64), C.c_int, C.POINTER(C.c_int)]),
    "dfmm_server_create": (C.c_int, [C.POINTER(_P), C.c_int, C.c_size_t, C.c_int, C.c_int, C.POINTER(_P)]),
    "dfmm_server_submit": (C.c_int, [_P, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int64)]),
    "dfmm_server_wait": (C.c_int, [_P, C.c_int64, _D, _D]),
    "dfmm_server_drain": (C.c_int, [_P]),
    "dfmm_server_now": (C.c_double, [_P]),
    "dfmm_server_passes": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "dfmm_server_pass": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "dfmm_server_footprint": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "dfmm_server_destroy": (None, [_P]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class DfmmError(RuntimeError):
    def __init__(self, status: int):
        self.status = status
        name = _lib.dfmm_status_string(status).decode()
        detail = _lib.dfmm_last_error().decode()
        super().__init__(f"{name}: {detail}")


def _check(status: int) -> None:
    if status != 0:
        raise DfmmError(status)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


class OpSet:
    """Directional skeletons (a, b, D) of Eq. 2 for widths 1/2 (LF) and 1 .. w_hi."""

    def __init__(self, handle):
        self._h = _P(handle)

    @classmethod
    def build(cls, tau: float, w_hi: int, cache_dir: str | None = None) -> "OpSet":
        h = _P()
        _check(_lib.dfmm_opset_build(tau, w_hi, cache_dir.encode() if cache_dir else None, C.byref(h)))
        return cls(h.value)

    @classmethod
    def create(cls, tau: float, w_hi: int) -> "OpSet":
        h = _P()
        _check(_lib.dfmm_opset_create(tau, w_hi, C.byref(h)))
        return cls(h.value)

    @classmethod
    def load(cls, path: str) -> "OpSet":
        h = _P()
        _check(_lib.dfmm_opset_load(path.encode(), C.byref(h)))
        return cls(h.value)

    def save(self, path: str) -> None:
        _check(_lib.dfmm_opset_save(self._h, path.encode()))

    def set(self, w: float, d: int, a, b, D) -> None:
        a = np.ascontiguousarray(a, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        Dm = np.ascontiguousarray(np.asarray(D, dtype=np.complex128)).view(np.float64)
        r = a.shape[0]
        _check(_lib.dfmm_opset_set(self._h, float(w), int(d), r, _dptr(a), _dptr(b), _dptr(Dm)))

    def get(self, w: float, d: int):
        r = C.c_int()
        _check(_lib.dfmm_opset_get(self._h, float(w), int(d), C.byref(r), None, None, None))
        n = r.value
        a = np.empty((n, 3))
        b = np.empty((n, 3))
        D = np.empty((n, n), dtype=np.complex128)
        _check(_lib.dfmm_opset_get(self._h, float(w), int(d), C.byref(r), _dptr(a), _dptr(b),
                                   D.view(np.float64).ctypes.data_as(_D)))
        return a, b, D

    def info(self):
        tau = C.c_double()
        w = C.c_int()
        _check(_lib.dfmm_opset_info(self._h, C.byref(tau), C.byref(w)))
        return tau.value, w.value

    def close(self) -> None:
        if self._h:
            _lib.dfmm_opset_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A resident plan for one point set: dfmm_plan / dfmm_plan_ex."""

    def __init__(self, points, K: float, eps: float = 1e-4, opset: OpSet | None = None,
                 cache_dir: str | None = None, device: int = -1, precision: int = 0,
                 leaf_width: float = 0.0, tol_factor: float = 0.0, hbm_budget_bytes: int = 0,
                 leaf_max: int = 0, lf_levels: int = 0):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2 or pts.shape[1] != 3:
            raise ValueError("points must be (N, 3)")
        opt = Options()
        _lib.dfmm_options_default(C.byref(opt))
        opt.eps = eps
        opt.opset = opset._h.value if opset is not None else None
        self._cache = cache_dir.encode() if cache_dir else None
        opt.cache_dir = self._cache
        opt.device = device
        opt.precision = precision
        opt.leaf_width = leaf_width
        opt.tol_factor = tol_factor
        opt.hbm_budget_bytes = hbm_budget_bytes
        opt.leaf_max = leaf_max
        opt.lf_levels = lf_levels
        h = _P()
        _check(_lib.dfmm_plan_ex(_dptr(pts), pts.shape[0], float(K), C.byref(opt), C.byref(h)))
        self._h = h
        self.N = pts.shape[0]
        self.K = K
        self.precision = precision

    def _ctype(self):
        import torch

        return torch.complex128 if self.precision == PREC_FP64 else torch.complex64

    def apply(self, f, u=None, stream=None):
        """u = A f for a (nrhs, N) CUDA tensor f (or (N,)): complex64, or complex128
        for float64 plans; returns u."""
        import torch

        one = f.dim() == 1
        f2 = f.reshape(1, -1) if one else f
        if f2.dtype != self._ctype() or not f2.is_cuda or not f2.is_contiguous():
            raise ValueError(f"f must be a contiguous {self._ctype()} CUDA tensor")
        if f2.shape[1] != self.N:
            raise ValueError("f has the wrong number of points")
        if u is None:
            u = torch.empty_like(f2)
        if stream is None:
            stream = torch.cuda.current_stream(f2.device)
        _check(_lib.dfmm_apply(self._h, C.c_void_p(f2.data_ptr()), C.c_void_p(u.data_ptr()),
                               f2.shape[0], C.c_void_p(stream.cuda_stream)))
        return u.reshape(-1) if one else u

    def apply_ws(self, f, u, ws, stream=None):
        """dfmm_apply_ws: u = A f with the caller's workspace ws (a CUDA tensor of at
        least workspace_bytes(nrhs) bytes, 256-byte aligned); everything runs on
        ``stream`` (default: the current stream)."""
        import torch

        one = f.dim() == 1
        f2 = f.reshape(1, -1) if one else f
        if f2.dtype != self._ctype() or not f2.is_cuda or not f2.is_contiguous() or f2.shape[1] != self.N:
            raise ValueError(f"f must be a contiguous (nrhs, N) {self._ctype()} CUDA tensor")
        u2 = u.reshape(f2.shape)
        if u2.dtype != f2.dtype or not u2.is_contiguous():
            raise ValueError("u must be a contiguous tensor shaped and typed like f")
        if not ws.is_cuda or not ws.is_contiguous():
            raise ValueError("ws must be a contiguous CUDA tensor")
        if stream is None:
            stream = torch.cuda.current_stream(f2.device)
        nbytes = ws.numel() * ws.element_size()
        _check(_lib.dfmm_apply_ws(self._h, C.c_void_p(f2.data_ptr()), C.c_void_p(u2.data_ptr()), f2.shape[0],
                                  C.c_void_p(ws.data_ptr()), nbytes, C.c_void_p(stream.cuda_stream)))
        return u

    def apply_noalloc(self, f, u, stream=None):
        """dfmm_apply_noalloc: u = A f on the library's static device workspace
        (no allocation); needs an earlier apply with the same nrhs."""
        import torch

        f2 = f.reshape(1, -1) if f.dim() == 1 else f
        if f2.dtype != torch.complex64 or not f2.is_cuda or not f2.is_contiguous() or f2.shape[1] != self.N:
            raise ValueError("f must be a contiguous (nrhs, N) complex64 CUDA tensor")
        u2 = u.reshape(f2.shape)
        if u2.dtype != torch.complex64 or not u2.is_contiguous():
            raise ValueError("u must be a contiguous complex64 tensor shaped like f")
        if stream is None:
            stream = torch.cuda.current_stream(f2.device)
        _check(_lib.dfmm_apply_noalloc(self._h, C.c_void_p(f2.data_ptr()), C.c_void_p(u2.data_ptr()),
                                       f2.shape[0], C.c_void_p(stream.cuda_stream)))
        return u

    def apply_batch(self, fs, us, stream=None):
        """One pass over several requests: us[r] = A fs[r] for (nrhs_r, N) complex64
        CUDA tensors (at most MAX_BATCH requests)."""
        import torch

        if len(fs) != len(us) or not 1 <= len(fs) <= MAX_BATCH:
            raise ValueError(f"need 1 .. {MAX_BATCH} (f, u) pairs")
        for f, u in zip(fs, us):
            if f.dtype != torch.complex64 or not f.is_cuda or not f.is_contiguous() or f.dim() != 2:
                raise ValueError("each f must be a contiguous (nrhs, N) complex64 CUDA tensor")
            if f.shape[1] != self.N or u.shape != f.shape or u.dtype != f.dtype or not u.is_contiguous():
                raise ValueError("request shapes do not match the plan")
        n = len(fs)
        fp = (C.c_void_p * n)(*[f.data_ptr() for f in fs])
        up = (C.c_void_p * n)(*[u.data_ptr() for u in us])
        nr = (C.c_int * n)(*[f.shape[0] for f in fs])
        if stream is None:
            stream = torch.cuda.current_stream(fs[0].device)
        _check(_lib.dfmm_apply_batch(self._h, n, fp, up, nr, C.c_void_p(stream.cuda_stream)))
        return us

    def workspace_bytes(self, nrhs: int) -> int:
        b = C.c_size_t()
        _check(_lib.dfmm_workspace_bytes(self._h, nrhs, C.byref(b)))
        return b.value

    def info(self) -> Info:
        inf = Info()
        _check(_lib.dfmm_plan_info(self._h, C.byref(inf)))
        return inf

    def export(self, what: int, level: int = 0) -> np.ndarray:
        n = C.c_size_t()
        _check(_lib.dfmm_export(self._h, what, level, None, C.byref(n)))
        buf = np.empty(n.value // 8, dtype=np.int64)
        _check(_lib.dfmm_export(self._h, what, level, buf.ctypes.data_as(C.c_void_p), C.byref(n)))
        width = {EXPORT_PERM: 1, EXPORT_BOXES: 5, EXPORT_PAIRS: 5, EXPORT_NEAR: 2,
                 EXPORT_OUT_SLOTS: 2, EXPORT_IN_SLOTS: 2, EXPORT_LEAVES: 4}[what]
        return buf if width == 1 else buf.reshape(-1, width)

    def set_timing(self, applies: int) -> None:
        """Record stage events for up to ``applies`` following applies (0 = off)."""
        _check(_lib.dfmm_set_timing(self._h, int(applies)))

    def stage_times(self) -> dict:
        """Summed ms and launch counts per stage over the recorded applies."""
        ms = (C.c_double * 16)()
        cnt = (C.c_int64 * 16)()
        n = C.c_int()
        _check(_lib.dfmm_stage_times(self._h, ms, cnt, 16, C.byref(n)))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES[: n.value])}

    def close(self) -> None:
        if self._h:
            _lib.dfmm_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A continuous-batching request loop over resident plans (dfmm_server_*):
    one stream per plan and a native worker thread that starts each plan's
    next pass when its previous one has finished.  Blocking calls release the
    GIL."""

    def __init__(self, plans, budget_bytes: int, max_batch_rhs: int = 32, single: bool = False):
        self.plans = list(plans)
        arr = (_P * len(self.plans))(*[p._h.value for p in self.plans])
        h = _P()
        _check(_lib.dfmm_server_create(arr, len(self.plans), int(budget_bytes), int(max_batch_rhs),
                                       int(bool(single)), C.byref(h)))
        self._h = h

    def submit(self, plan: int, f, u) -> int:
        """Queue u = A f for plan index ``plan`` ((nrhs, N) complex64 CUDA tensors;
        f must hold its values already); returns the request's ticket."""
        import torch

        if not 0 <= plan < len(self.plans):
            raise ValueError("no such plan")
        N = self.plans[plan].N
        if f.dtype != torch.complex64 or not f.is_cuda or not f.is_contiguous() or f.dim() != 2 or f.shape[1] != N:
            raise ValueError("f must be a contiguous (nrhs, N) complex64 CUDA tensor")
        if u.shape != f.shape or u.dtype != f.dtype or not u.is_contiguous():
            raise ValueError("u must be a contiguous tensor shaped and typed like f")
        t = C.c_int64()
        _check(_lib.dfmm_server_submit(self._h, plan, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                       f.shape[0], C.byref(t)))
        return t.value

    def wait(self, ticket: int):
        """Blocks until the request has finished; returns (t_submit, t_done) in
        seconds on the server's clock, or raises DfmmError with its status."""
        a, b = C.c_double(), C.c_double()
        _check(_lib.dfmm_server_wait(self._h, int(ticket), C.byref(a), C.byref(b)))
        return a.value, b.value

    def drain(self) -> None:
        _check(_lib.dfmm_server_drain(self._h))

    def now(self) -> float:
        return _lib.dfmm_server_now(self._h)

    def passes(self) -> list:
        """(plan, requests, nrhs) of every pass started so far, in order."""
        n = C.c_int64()
        _check(_lib.dfmm_server_passes(self._h, C.byref(n)))
        out = []
        p, q, k = C.c_int(), C.c_int(), C.c_int()
        for i in range(n.value):
            _check(_lib.dfmm_server_pass(self._h, i, C.byref(p), C.byref(q), C.byref(k)))
            out.append((p.value, q.value, k.value))
        return out

    def footprint(self) -> int:
        b = C.c_size_t()
        _check(_lib.dfmm_server_footprint(self._h, C.byref(b)))
        return b.value

    def close(self) -> None:
        """Waits for every submitted request, then frees the server."""
        if self._h:
            _lib.dfmm_server_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def status_string(s: int) -> str:
    return _lib.dfmm_status_string(s).decode()
