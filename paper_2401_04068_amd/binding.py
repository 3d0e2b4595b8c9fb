"""ctypes binding of liblti_freqresp.so (argument marshalling only).

Every step of the computation runs in the HIP library; this module only
builds the C structs, keeps the caller's buffers alive while a request is in
flight, and converts results to numpy / torch.  PyTorch provides the device
arena (one ``torch.empty(..., dtype=uint8, device='cuda')`` tensor that the
library sub-allocates) and, optionally, the stream.

There is no fallback: if the shared library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Any, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblti_freqresp.so")

ABI_VERSION = 4

LTI_OK = 0
LTI_PENDING = 1
LTI_EINVAL = -1
LTI_ENOSPC = -2
LTI_EAGAIN = -3
LTI_ENOENT = -4
LTI_EDEVICE = -5
LTI_ENOMEM = -6
LTI_EUNSUPPORTED = -7

PREC_FP64 = 0
PREC_REFINED = 1
MEM_HOST = 0
MEM_DEVICE = 1

PATH_FP64 = 0
PATH_REFINED = 1
PATH_FALLBACK = 2
PATH_SINGULAR = 3
PATH_FP64_DD = 4

POINTS_JW = 0
POINTS_S = 1
POINTS_Z = 2

KF_SWEEP4 = 0
KF_SWEEP1 = 1
KF_SWEEPWG = 2
KF_REFINE_DD = 3
KF_SWEEPDESC = 4
KF_SWEEP2 = 5
KF_COUNT = 6

CFG_KERNEL_TIMING = 1
CFG_FORCE_DD = 2
CFG_NO_TRANSPOSE = 4

POINT_INFO_DTYPE = np.dtype(
    [("est_rel_err", "<f4"), ("iters", "u1"), ("path", "u1"), ("reserved", "<u2")]
)

# Every symbol the header declares; checked by the CPU test-suite.
EXPORTS = (
    "lti_freqresp_create",
    "lti_freqresp_submit",
    "lti_freqresp_poll",
    "lti_freqresp_destroy",
    "lti_freqresp_get_reduced",
    "lti_freqresp_stats",
    "lti_freqresp_strerror",
    "lti_freqresp_abi_version",
    "lti_freqresp_peaks",
    "lti_freqresp_eval_noalloc",
)


class LtiConfig(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("device", ctypes.c_int32),
        ("arena", ctypes.c_void_p),
        ("arena_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("max_pending", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("tile_points", ctypes.c_int32),
        ("max_batch_tiles", ctypes.c_int32),
        ("host_staging_bytes", ctypes.c_size_t),
    ]


class LtiRequest(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("nu", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("mem", ctypes.c_int32),
        ("A", ctypes.c_void_p),
        ("B", ctypes.c_void_p),
        ("C", ctypes.c_void_p),
        ("D", ctypes.c_void_p),
        ("omega", ctypes.c_void_p),
        ("n_omega", ctypes.c_int64),
        ("precision", ctypes.c_int32),
        ("points", ctypes.c_int32),
        ("rtol", ctypes.c_double),
        ("model_key", ctypes.c_uint64),
        ("G_out", ctypes.c_void_p),
        ("info_out", ctypes.c_void_p),
        ("dG_out", ctypes.c_void_p),
        ("E", ctypes.c_void_p),
    ]


class LtiResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("reduction_reused", ctypes.c_int32),
        ("n_points", ctypes.c_int64),
        ("n_refined", ctypes.c_int64),
        ("n_fallback", ctypes.c_int64),
        ("n_singular", ctypes.c_int64),
        ("n_fp64_dd", ctypes.c_int64),
        ("max_est_rel_err", ctypes.c_double),
        ("t_submit_us", ctypes.c_double),
        ("t_admit_us", ctypes.c_double),
        ("t_first_launch_us", ctypes.c_double),
        ("t_done_us", ctypes.c_double),
    ]


class LtiPeak(ctypes.Structure):
    _fields_ = [("w", ctypes.c_double), ("gain", ctypes.c_double)]


class LtiHinfResult(ctypes.Structure):
    _fields_ = [("hinf", ctypes.c_double), ("w_hinf", ctypes.c_double), ("n_peaks", ctypes.c_int32),
                ("evaluations", ctypes.c_int32)]


class LtiStats(ctypes.Structure):
    _fields_ = [
        ("requests_submitted", ctypes.c_uint64),
        ("requests_done", ctypes.c_uint64),
        ("requests_failed", ctypes.c_uint64),
        ("reductions", ctypes.c_uint64),
        ("reduction_cache_hits", ctypes.c_uint64),
        ("sweep_launches", ctypes.c_uint64),
        ("tiles_launched", ctypes.c_uint64),
        ("points_done", ctypes.c_uint64),
        ("arena_bytes_in_use", ctypes.c_uint64),
        ("arena_peak_bytes", ctypes.c_uint64),
        ("sweep_kernel_ms", ctypes.c_double),
        ("reduce_kernel_ms", ctypes.c_double),
        ("timed_sweep_launches", ctypes.c_uint64),
        ("timed_reduce_launches", ctypes.c_uint64),
        ("family_ms", ctypes.c_double * KF_COUNT),
        ("family_launches", ctypes.c_uint64 * KF_COUNT),
    ]


# imdp_vi.h: robust value iteration for interval MDPs
IMDP_EXPORTS = ("imdp_vi_create", "imdp_vi_run", "imdp_vi_destroy")
IMDP_OK = 0
IMDP_EINVAL = -1
IMDP_EDEVICE = -5
IMDP_ENOMEM = -6
IMDP_EUNSUPPORTED = -7
IMDP_REACH = 0
IMDP_REACH_AVOID = 1
IMDP_REWARD = 2


class ImdpModel(ctypes.Structure):
    _fields_ = [
        ("n_states", ctypes.c_int32),
        ("n_columns", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("stateptr", ctypes.c_void_p),
        ("colptr", ctypes.c_void_p),
        ("rowval", ctypes.c_void_p),
        ("lower", ctypes.c_void_p),
        ("upper", ctypes.c_void_p),
    ]


class ImdpSpec(ctypes.Structure):
    _fields_ = [
        ("property", ctypes.c_int32),
        ("horizon", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("max_iterations", ctypes.c_int32),
        ("pessimistic", ctypes.c_int32),
        ("maximize", ctypes.c_int32),
        ("targets", ctypes.c_void_p),
        ("n_targets", ctypes.c_int32),
        ("avoid", ctypes.c_void_p),
        ("n_avoid", ctypes.c_int32),
        ("reward", ctypes.c_void_p),
        ("discount", ctypes.c_double),
    ]


class ImdpResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("residual", ctypes.c_double), ("kernel_ms", ctypes.c_double)]


_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the shared library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2401_04068_amd.build` "
            "(there is no CPU fallback)"
        )
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.lti_freqresp_create.argtypes = [P(LtiConfig), P(ctypes.c_void_p)]
    lib.lti_freqresp_create.restype = ctypes.c_int
    lib.lti_freqresp_submit.argtypes = [ctypes.c_void_p, P(LtiRequest), P(ctypes.c_uint64)]
    lib.lti_freqresp_submit.restype = ctypes.c_int
    lib.lti_freqresp_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, P(LtiResult)]
    lib.lti_freqresp_poll.restype = ctypes.c_int
    lib.lti_freqresp_destroy.argtypes = [ctypes.c_void_p]
    lib.lti_freqresp_destroy.restype = ctypes.c_int
    lib.lti_freqresp_get_reduced.argtypes = [
        ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
    ]
    lib.lti_freqresp_get_reduced.restype = ctypes.c_int
    lib.lti_freqresp_stats.argtypes = [ctypes.c_void_p, P(LtiStats)]
    lib.lti_freqresp_stats.restype = ctypes.c_int
    lib.lti_freqresp_strerror.argtypes = [ctypes.c_int]
    lib.lti_freqresp_strerror.restype = ctypes.c_char_p
    lib.lti_freqresp_peaks.argtypes = [ctypes.c_void_p, P(LtiRequest), ctypes.c_int32, ctypes.c_double,
                                       P(LtiPeak), P(LtiHinfResult)]
    lib.lti_freqresp_peaks.restype = ctypes.c_int
    lib.lti_freqresp_eval_noalloc.argtypes = [ctypes.c_int32, P(LtiRequest), ctypes.c_void_p]
    lib.lti_freqresp_eval_noalloc.restype = ctypes.c_int
    lib.imdp_vi_create.argtypes = [ctypes.c_int32, P(ImdpModel), P(ctypes.c_void_p)]
    lib.imdp_vi_create.restype = ctypes.c_int
    lib.imdp_vi_run.argtypes = [ctypes.c_void_p, P(ImdpSpec), ctypes.c_void_p, ctypes.c_void_p, P(ImdpResult)]
    lib.imdp_vi_run.restype = ctypes.c_int
    lib.imdp_vi_destroy.argtypes = [ctypes.c_void_p]
    lib.imdp_vi_destroy.restype = ctypes.c_int
    lib.lti_freqresp_abi_version.argtypes = []
    lib.lti_freqresp_abi_version.restype = ctypes.c_uint32
    if lib.lti_freqresp_abi_version() != ABI_VERSION:
        raise ImportError("liblti_freqresp.so ABI version mismatch; rebuild it")
    _lib = lib
    return lib


def eval_noalloc(A, B, C, D, omega, G, info=None, precision: int = PREC_FP64, rtol: float = 0.0,
                 points: int = POINTS_JW, dG=None, device: int = 0, stream=None) -> None:
    """lti_freqresp_eval_noalloc: enqueue one device-memory evaluation on
    `stream` (default: torch's current stream on `device`) that allocates
    nothing; the results are ready once that stream reaches this point.
    Arguments as for Engine.submit_device."""
    import torch

    lib = load()
    for t in (A, B, C, omega):
        if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("device inputs must be contiguous float64 CUDA tensors")
    req = LtiRequest()
    req.nx, req.nu, req.ny = A.shape[0], B.shape[1], C.shape[0]
    req.mem = MEM_DEVICE
    req.A, req.B, req.C = A.data_ptr(), B.data_ptr(), C.data_ptr()
    req.D = None if D is None else D.data_ptr()
    req.omega = omega.data_ptr()
    req.n_omega = omega.numel() // (2 if points == POINTS_S else 1)
    req.precision = int(precision)
    req.points = int(points)
    req.rtol = float(rtol)
    req.G_out = G.data_ptr()
    req.info_out = None if info is None else info.data_ptr()
    req.dG_out = None if dG is None else dG.data_ptr()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    rc = lib.lti_freqresp_eval_noalloc(int(device), ctypes.byref(req), ctypes.c_void_p(stream.cuda_stream))
    if rc != LTI_OK:
        raise LtiError(rc, "lti_freqresp_eval_noalloc")


def strerror(code: int) -> str:
    return load().lti_freqresp_strerror(int(code)).decode()


class LtiError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


@dataclass
class Handle:
    id: int
    G: Any  # numpy (K, p, m) complex128 view, or device tensor
    info: Any
    keep: list = field(default_factory=list)
    result: Optional[dict] = None
    dG: Any = None  # dG/ds, when requested


def _result_dict(r: LtiResult) -> dict:
    return {name: getattr(r, name) for name, _ in LtiResult._fields_}


class Engine:
    """One library context on one device, with its arena from PyTorch."""

    def __init__(
        self,
        arena_bytes: int = 1 << 30,
        device: int = 0,
        stream=None,
        kernel_timing: bool = False,
        tile_points: int = 0,
        max_batch_tiles: int = 0,
        max_pending: int = 0,
        host_staging_bytes: int = 0,
        flags: int = 0,
    ):
        import torch

        lib = load()
        self._torch = torch
        self.device = device
        self._arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self._stream = stream
        cfg = LtiConfig()
        cfg.abi_version = ABI_VERSION
        cfg.device = device
        cfg.arena = self._arena.data_ptr()
        cfg.arena_bytes = int(arena_bytes)
        cfg.stream = stream.cuda_stream if stream is not None else None
        cfg.max_pending = max_pending
        cfg.flags = (CFG_KERNEL_TIMING if kernel_timing else 0) | int(flags)
        cfg.tile_points = tile_points
        cfg.max_batch_tiles = max_batch_tiles
        cfg.host_staging_bytes = host_staging_bytes
        ctx = ctypes.c_void_p()
        rc = lib.lti_freqresp_create(ctypes.byref(cfg), ctypes.byref(ctx))
        if rc != LTI_OK:
            raise LtiError(rc, "lti_freqresp_create")
        self._ctx = ctx
        self._lib = lib

    # ------------------------------------------------------------ requests
    def submit(self, A, B, C, D, omega, precision: int = PREC_FP64, model_key: int = 0,
               rtol: float = 0.0, want_info: bool = True, points: int = POINTS_JW,
               want_derivative: bool = False, E=None, out=None) -> Handle:
        """Host-memory request; inputs are copied before this returns.

        points: POINTS_JW (omega real, s = j omega), POINTS_S (omega complex
        points s), POINTS_Z (omega = theta in rad/sample, z = exp(j theta)).
        out: optional (G, info) host arrays to receive the results (G
        complex128 (K, p, m), info POINT_INFO_DTYPE (K,) or None), e.g. buffers
        a caller reuses; by default new arrays are allocated."""
        A, B, C = _f64(A), _f64(B), _f64(C)
        n, m, p = A.shape[0], B.shape[1], C.shape[0]
        Dm = None if D is None else _f64(D)
        if points == POINTS_S:
            w = np.ascontiguousarray(np.asarray(omega, dtype=np.complex128).reshape(-1)).view(np.float64)
            K = w.shape[0] // 2
        else:
            w = _f64(omega).reshape(-1)
            K = w.shape[0]
        if out is None:
            G = np.empty((K, p, m), dtype=np.complex128)
            info = np.zeros(K, dtype=POINT_INFO_DTYPE) if want_info else None
        else:
            G, info = out
            if (not isinstance(G, np.ndarray) or G.dtype != np.complex128 or G.shape != (K, p, m)
                    or not G.flags.c_contiguous):
                raise ValueError("out G must be a C-contiguous complex128 array of shape (K, p, m)")
            if info is not None and (not isinstance(info, np.ndarray) or info.dtype != POINT_INFO_DTYPE
                                     or info.shape != (K,) or not info.flags.c_contiguous):
                raise ValueError("out info must be a C-contiguous POINT_INFO_DTYPE array of shape (K,)")
        req = LtiRequest()
        req.nx, req.nu, req.ny = n, m, p
        req.mem = MEM_HOST
        req.A, req.B, req.C = A.ctypes.data, B.ctypes.data, C.ctypes.data
        req.D = None if Dm is None else Dm.ctypes.data
        req.omega = w.ctypes.data
        req.n_omega = K
        req.precision = int(precision)
        req.points = int(points)
        req.rtol = float(rtol)
        req.model_key = int(model_key)
        req.G_out = G.ctypes.data
        req.info_out = None if info is None else info.ctypes.data
        dG = np.empty((K, p, m), dtype=np.complex128) if want_derivative else None
        req.dG_out = None if dG is None else dG.ctypes.data
        Em = None if E is None else _f64(E)
        req.E = None if Em is None else Em.ctypes.data
        rid = ctypes.c_uint64()
        rc = self._lib.lti_freqresp_submit(self._ctx, ctypes.byref(req), ctypes.byref(rid))
        if rc != LTI_OK:
            raise LtiError(rc, "lti_freqresp_submit")
        return Handle(rid.value, G, info, keep=[G, info, dG], dG=dG)

    def submit_device(self, A, B, C, D, omega, G, info=None, precision: int = PREC_FP64,
                      model_key: int = 0, rtol: float = 0.0, points: int = POINTS_JW, dG=None, E=None) -> Handle:
        """Device-memory request: torch float64 tensors on this engine's device;
        G is a float64 tensor of 2*K*p*m entries (or complex128 (K, p, m)).
        Nothing is copied; the tensors must stay alive and unmodified until
        the request is done."""
        torch = self._torch
        for t in (A, B, C, omega):
            if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
                raise ValueError("device inputs must be contiguous float64 CUDA tensors")
        n, m, p = A.shape[0], B.shape[1], C.shape[0]
        req = LtiRequest()
        req.nx, req.nu, req.ny = n, m, p
        req.mem = MEM_DEVICE
        req.A, req.B, req.C = A.data_ptr(), B.data_ptr(), C.data_ptr()
        req.D = None if D is None else D.data_ptr()
        req.omega = omega.data_ptr()
        req.n_omega = omega.numel() // (2 if points == POINTS_S else 1)
        req.precision = int(precision)
        req.points = int(points)
        req.rtol = float(rtol)
        req.model_key = int(model_key)
        req.G_out = G.data_ptr()
        req.info_out = None if info is None else info.data_ptr()
        req.dG_out = None if dG is None else dG.data_ptr()
        req.E = None if E is None else E.data_ptr()
        rid = ctypes.c_uint64()
        rc = self._lib.lti_freqresp_submit(self._ctx, ctypes.byref(req), ctypes.byref(rid))
        if rc != LTI_OK:
            raise LtiError(rc, "lti_freqresp_submit")
        return Handle(rid.value, G, info, keep=[A, B, C, D, omega, G, info, dG, E], dG=dG)

    def poll(self, h: Handle, timeout_us: int = -1) -> bool:
        """True when done (result in h.result); False while pending."""
        res = LtiResult()
        rc = self._lib.lti_freqresp_poll(self._ctx, h.id, int(timeout_us), ctypes.byref(res))
        if rc == LTI_PENDING:
            return False
        if rc != LTI_OK:
            raise LtiError(rc, "lti_freqresp_poll")
        h.result = _result_dict(res)
        h.keep = []
        return True

    def wait(self, h: Handle) -> Handle:
        self.poll(h, -1)
        return h

    def peaks(self, A, B, C, D, omega, max_peaks: int = 8, wtol: float = 1e-12):
        """lti_freqresp_peaks: resonance peaks [(w, gain), ...] (largest
        first) and {'hinf', 'w_hinf', 'n_peaks', 'evaluations'}."""
        A, B, C = _f64(A), _f64(B), _f64(C)
        Dm = None if D is None else _f64(D)
        w = _f64(omega).reshape(-1)
        req = LtiRequest()
        req.nx, req.nu, req.ny = A.shape[0], B.shape[1], C.shape[0]
        req.mem = MEM_HOST
        req.A, req.B, req.C = A.ctypes.data, B.ctypes.data, C.ctypes.data
        req.D = None if Dm is None else Dm.ctypes.data
        req.omega = w.ctypes.data
        req.n_omega = w.shape[0]
        req.precision = PREC_FP64
        req.points = POINTS_JW
        req.G_out = w.ctypes.data  # not written: the call evaluates into its own buffers
        out = LtiHinfResult()
        pk = (LtiPeak * max(1, max_peaks))()
        rc = self._lib.lti_freqresp_peaks(self._ctx, ctypes.byref(req), int(max_peaks), float(wtol), pk,
                                          ctypes.byref(out))
        if rc != LTI_OK:
            raise LtiError(rc, "lti_freqresp_peaks")
        peaks = [(pk[i].w, pk[i].gain) for i in range(out.n_peaks)]
        return peaks, {name: getattr(out, name) for name, _ in LtiHinfResult._fields_}

    # ------------------------------------------------------------ helpers
    def stats(self) -> dict:
        s = LtiStats()
        rc = self._lib.lti_freqresp_stats(self._ctx, ctypes.byref(s))
        if rc != LTI_OK:
            raise LtiError(rc, "lti_freqresp_stats")
        out = {name: getattr(s, name) for name, _ in LtiStats._fields_}
        out["family_ms"] = list(s.family_ms)
        out["family_launches"] = list(s.family_launches)
        return out

    def get_reduced(self, model_key: int, n: int, m: int, p: int):
        H = np.empty((n, n))
        Bt = np.empty((n, m))
        Ct = np.empty((p, n))
        rc = self._lib.lti_freqresp_get_reduced(self._ctx, int(model_key), n, m, p,
                                                H.ctypes.data, Bt.ctypes.data, Ct.ctypes.data)
        if rc != LTI_OK:
            raise LtiError(rc, "lti_freqresp_get_reduced")
        return H, Bt, Ct

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lti_freqresp_destroy(self._ctx)
            self._ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def freqresp(A, B, C, D, omega, precision: int = PREC_FP64, engine: Optional[Engine] = None,
             model_key: int = 0):
    """Convenience: one synchronous request.  Returns (G (K, p, m) complex128, info)."""
    own = engine is None
    eng = engine or Engine(arena_bytes=256 << 20)
    try:
        h = eng.submit(A, B, C, D, omega, precision=precision, model_key=model_key)
        eng.wait(h)
        return h.G, h.info
    finally:
        if own:
            eng.close()


class ImdpError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: error {code}")


def _i32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


class IMDPSolver:
    """imdp_vi_create / _run / _destroy: an interval MDP in compressed sparse
    columns (one column per state-action pair) copied to the device once,
    then value iteration runs against it."""

    def __init__(self, n_states, stateptr, colptr, rowval, lower, upper, device: int = 0):
        lib = load()
        self._lib = lib
        self._keep = [_i32(stateptr), _i32(colptr), _i32(rowval), _f64(lower), _f64(upper)]
        sp, cp, rv, lo, up = self._keep
        m = ImdpModel()
        m.n_states = int(n_states)
        m.n_columns = len(cp) - 1
        m.nnz = len(rv)
        m.stateptr, m.colptr, m.rowval = sp.ctypes.data, cp.ctypes.data, rv.ctypes.data
        m.lower, m.upper = lo.ctypes.data, up.ctypes.data
        h = ctypes.c_void_p()
        rc = lib.imdp_vi_create(int(device), ctypes.byref(m), ctypes.byref(h))
        self._keep = []  # copied by the library
        if rc != IMDP_OK:
            raise ImdpError(rc, "imdp_vi_create")
        self._h = h
        self.n_states = int(n_states)

    def run(self, prop: int = IMDP_REACH, horizon: int = 100, eps: float = 1e-6, targets=(), avoid=(),
            reward=None, discount: float = 1.0, pessimistic: bool = True, maximize: bool = True,
            want_policy: bool = True, max_iterations: int = 0):
        """Returns (V, iterations, residual, policy, kernel_ms); policy is
        (n_states, horizon) for a finite horizon, (n_states,) otherwise."""
        t = _i32(targets)
        a = _i32(avoid)
        r = None if reward is None else _f64(reward)
        spec = ImdpSpec()
        spec.property = int(prop)
        spec.horizon = int(horizon)
        spec.eps = float(eps)
        spec.max_iterations = int(max_iterations)
        spec.pessimistic = 1 if pessimistic else 0
        spec.maximize = 1 if maximize else 0
        spec.targets = t.ctypes.data if len(t) else None
        spec.n_targets = len(t)
        spec.avoid = a.ctypes.data if len(a) else None
        spec.n_avoid = len(a)
        spec.reward = None if r is None else r.ctypes.data
        spec.discount = float(discount)
        V = np.empty(self.n_states)
        pol = None
        if want_policy:
            pol = np.empty((self.n_states, horizon) if horizon > 0 else (self.n_states,), dtype=np.int32)
        res = ImdpResult()
        rc = self._lib.imdp_vi_run(self._h, ctypes.byref(spec), V.ctypes.data,
                                   None if pol is None else pol.ctypes.data, ctypes.byref(res))
        if rc != IMDP_OK:
            raise ImdpError(rc, "imdp_vi_run")
        return V, res.iterations, res.residual, pol, res.kernel_ms

    def close(self):
        if getattr(self, "_h", None):
            self._lib.imdp_vi_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
