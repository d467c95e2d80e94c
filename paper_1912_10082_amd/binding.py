"""ctypes binding of the C ABI in include/sts.h (argument marshalling only).

Every computation runs in ``libsts.so``; this module only converts arguments:
NumPy arrays are passed as host memory, PyTorch CUDA tensors as device memory
(column-major, float64), and PyTorch supplies device allocations and the
current stream.  If the library cannot be loaded the calls raise; there is no
other implementation to fall back to.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsts.so")

STS_OK, STS_E_INVALID, STS_E_NOMEM, STS_E_DEVICE, STS_E_NOT_CONVERGED, STS_E_NUMERIC, STS_E_STATE = range(7)
STATUS_NAMES = {0: "STS_OK", 1: "STS_E_INVALID", 2: "STS_E_NOMEM", 3: "STS_E_DEVICE",
                4: "STS_E_NOT_CONVERGED", 5: "STS_E_NUMERIC", 6: "STS_E_STATE"}
STS_MEM_HOST, STS_MEM_DEVICE = 0, 1
STS_FE_P1_1D, STS_FE_P1_2D, STS_FE_Q1_3D_7PT = 1, 2, 3
STS_OP_K, STS_OP_M = 0, 1
STS_K_COUNT = 21


class STSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Space(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("n", C.c_int64 * 3), ("mu", C.c_double)]


class Bidiag(C.Structure):
    _fields_ = [("diag", C.POINTER(C.c_double)), ("sub", C.POINTER(C.c_double))]


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_outer", C.c_int32), ("check_every", C.c_int32),
                ("inner_rtol", C.c_double), ("inner_maxit", C.c_int32), ("verify_true", C.c_int32),
                ("defl_tol", C.c_double), ("mem_budget", C.c_int64), ("restart", C.c_int32),
                ("profile", C.c_int32), ("inner_precond", C.c_int32), ("rational", C.c_int32),
                ("residual_qr", C.c_int32), ("inner_relax", C.c_int32),
                ("precond_fp32", C.c_int32), ("mixed", C.c_int32), ("orth_lag", C.c_int32),
                ("pad_", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("outer_its", C.c_int32), ("checks", C.c_int32), ("k", C.c_int64),
                ("rank", C.c_int64), ("inner_its_K", C.c_int64), ("inner_its_M", C.c_int64),
                ("res_cheap", C.c_double), ("res_true", C.c_double), ("orth_err", C.c_double),
                ("seconds", C.c_double), ("alg_bytes", C.c_double), ("breakdown", C.c_int32),
                ("shifts", C.c_int32), ("cg_poll_restarts", C.c_int64),
                ("res_floor", C.c_double), ("floor_limited", C.c_int32), ("pad_", C.c_int32),
                ("inner_its_fp32", C.c_int64), ("defect_rounds", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}


class Request(C.Structure):
    _fields_ = [("space", Space), ("nt", C.c_int64), ("p", C.c_int32), ("pad_", C.c_int32),
                ("dt_diag", C.POINTER(C.c_double)), ("dt_sub", C.POINTER(C.c_double)),
                ("mt_diag", C.POINTER(C.c_double)), ("mt_sub", C.POINTER(C.c_double)),
                ("F1", C.POINTER(C.c_double)), ("ldf1", C.c_int64),
                ("F2", C.POINTER(C.c_double)), ("ldf2", C.c_int64), ("opts", Opts)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("pad_", C.c_int32), ("queued_seconds", C.c_double),
                ("latency_seconds", C.c_double), ("footprint", C.c_int64), ("info", Info)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("released", C.c_int64),
                ("queued", C.c_int64), ("running", C.c_int64), ("mem_in_use", C.c_int64),
                ("mem_peak", C.c_int64), ("mem_budget", C.c_int64)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I64, _I32, _F64 = C.c_int64, C.c_int32, C.c_double

_SIGS = {
    "sts_default_opts": (None, [C.POINTER(Opts)]),
    "sts_last_error": (C.c_char_p, []),
    "sts_time_matrices": (C.c_int, [_I64, _D, _D, _D, _D, _D]),
    "sts_create": (C.c_int, [C.POINTER(Space), C.POINTER(Bidiag), C.POINTER(Bidiag), _I64, _I32,
                             _P, _I64, _P, _I64, _I32, _P, C.POINTER(_P)]),
    "sts_solve": (C.c_int, [_P, C.POINTER(Opts), C.POINTER(Info)]),
    "sts_rank": (C.c_int, [_P, C.POINTER(_I64)]),
    "sts_get_factors": (C.c_int, [_P, _P, _I64, _P, _I64, _I32, _P]),
    "sts_true_residual": (C.c_int, [_P, _D]),
    "sts_numerical_rank": (C.c_int, [_P, C.POINTER(_I64)]),
    "sts_destroy": (None, [_P]),
    "sts_release_cached_memory": (None, []),
    "sts_kernel_profile": (C.c_int, [_P, _I32, C.POINTER(_F64), C.POINTER(_I64), C.POINTER(_F64)]),
    "sts_kernel_name": (C.c_char_p, [_I32]),
    "sts_apply_op": (C.c_int, [C.POINTER(Space), _I32, _P, _I64, _P, _I64, _I32, _P]),
    "sts_cg": (C.c_int, [C.POINTER(Space), C.POINTER(_I32), _P, _I64, _P, _I64, _I32, _F64, _I32,
                         C.POINTER(_I32), _P]),
    "sts_pcg_mg": (C.c_int, [C.POINTER(Space), _P, _I64, _P, _I64, _I32, _F64, _I32,
                             C.POINTER(_I32), _P]),
    "sts_mg_vcycle": (C.c_int, [C.POINTER(Space), _P, _I64, _P, _I64, _I32, _P]),
    "sts_mg_vcycle_shifted": (C.c_int, [C.POINTER(Space), _F64, _P, _I64, _P, _I64, _I32, _P]),
    "sts_mg_vcycle_mixed": (C.c_int, [C.POINTER(Space), _F64, _P, _I64, _P, _I64, _I32, _P]),
    "sts_pcg_mg_mixed": (C.c_int, [C.POINTER(Space), _F64, _P, _I64, _P, _I64, _I32, _F64, _I32,
                                   C.POINTER(_I32), _P]),
    "sts_pcg_mg_refined": (C.c_int, [C.POINTER(Space), _P, _I64, _P, _I64, _I32, _F64, _I32,
                                     C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64), _P]),
    "sts_adaptive_shift": (C.c_int, [_D, _I32, _D, _I32, _F64, _F64, _I32, _D]),
    "sts_shifted_solve": (C.c_int, [C.POINTER(Space), _F64, _P, _I64, _P, _I64, _I32, _F64, _I32,
                                    C.POINTER(_I32), _P]),
    "sts_tridiag_solve": (C.c_int, [C.POINTER(Space), C.POINTER(_I32), _P, _I64, _P, _I64, _I32,
                                    _P]),
    "sts_mass_solve": (C.c_int, [C.POINTER(Space), _P, _I64, _P, _I64, _I32, _F64,
                                 C.POINTER(_I32), _P]),
    "sts_m_orthonormalize": (C.c_int, [C.POINTER(Space), _P, _P, _I64, _I64, _P, _P, _I64, _I32,
                                       _F64, C.POINTER(_I32), C.POINTER(_I32), _P]),
    "sts_gram": (C.c_int, [_I64, _I32, _I32, _P, _I64, _P, _I64, _P, _I64, _P]),
    "sts_solution_columns": (C.c_int, [_P, C.POINTER(_I64), _I32, _P, _I64, _I32, _P]),
    "sts_gram_noalloc": (C.c_int, [_I64, _I32, _I32, _P, _I64, _P, _I64, _P, _I64, _P]),
    "sts_basis_update": (C.c_int, [_I64, _I32, _I32, _P, _I64, _P, _I64, _P, _I64, _P]),
    "sts_gram_fp32": (C.c_int, [_I64, _I32, _I32, _P, _I64, _P, _I64, _P, _I64, _P]),
    "sts_sym_eig": (C.c_int, [_I64, _P, _I64, _P, _P, _I64, _P]),
    "sts_time_sweep": (C.c_int, [_I64, _I64, _I32, _P, _P, _I64, _P, _I64, _P, _I64,
                                 C.POINTER(Bidiag), C.POINTER(Bidiag), _P, _I64, _P]),
    "sts_pool_create": (C.c_int, [_I32, C.POINTER(_P)]),
    "sts_pool_workers": (C.c_int, [_P, C.POINTER(_I32)]),
    "sts_pool_solve": (C.c_int, [_P, _I32, C.POINTER(_P), C.POINTER(Opts), _I32, C.POINTER(Info),
                                 C.POINTER(C.c_int)]),
    "sts_pool_destroy": (None, [_P]),
    "sts_footprint": (C.c_int64, [C.POINTER(Space), _I64, _I32, C.POINTER(Opts)]),
    "sts_server_create": (C.c_int, [_I32, _I64, C.POINTER(_P)]),
    "sts_server_submit": (C.c_int, [_P, C.POINTER(Request), C.POINTER(_I64)]),
    "sts_server_wait": (C.c_int, [_P, _I64, _F64, C.POINTER(Result), C.POINTER(_P)]),
    "sts_server_release": (C.c_int, [_P, _I64]),
    "sts_server_get_stats": (C.c_int, [_P, C.POINTER(ServerStats)]),
    "sts_server_destroy": (None, [_P]),
}

EXPORTED = tuple(_SIGS)
_lib = None
_lock = threading.Lock()


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libsts.so (building it first if it is absent) and declare signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            from . import build as _build
            _build.build()
        lib = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _check(code: int):
    if code != STS_OK:
        raise STSError(code, load().sts_last_error().decode())


# ----------------------------------------------------------------------------
# array marshalling
# ----------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _stream_handle(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _host_colmajor(a) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return np.asfortranarray(a)


def dev_colmajor(t):
    """A float64 CUDA tensor viewed as a column-major matrix -> (tensor, ptr, ld).

    Returns a (possibly copied) tensor whose memory is column-major, so that
    t[i, j] lives at ptr + (i + j * ld) * 8.
    """
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 CUDA tensor")
    if t.dim() == 1:
        t = t[:, None]
    if t.stride(0) != 1 or (t.shape[1] > 1 and t.stride(1) < t.shape[0]):
        t = t.t().contiguous().t()
    ld = t.stride(1) if t.shape[1] > 1 else max(t.shape[0], 1)
    return t, C.c_void_p(t.data_ptr()), int(ld)


def dev_empty(rows: int, cols: int, device="cuda"):
    """Uninitialised column-major float64 CUDA matrix (rows x cols)."""
    torch = _torch()
    return torch.empty((cols, rows), dtype=torch.float64, device=device).t()


def dev_zeros(rows: int, cols: int, device="cuda"):
    torch = _torch()
    return torch.zeros((cols, rows), dtype=torch.float64, device=device).t()


def make_space(dim: int, n: int, mu: float = 1.0) -> Space:
    s = Space()
    s.kind = {1: STS_FE_P1_1D, 2: STS_FE_P1_2D, 3: STS_FE_Q1_3D_7PT}[dim]
    for d in range(3):
        s.n[d] = n if d < dim else 1
    s.mu = mu
    return s


def _bidiag(diag: np.ndarray, sub: np.ndarray):
    diag = np.ascontiguousarray(diag, dtype=np.float64)
    sub = np.ascontiguousarray(sub, dtype=np.float64)
    b = Bidiag(diag.ctypes.data_as(_D), sub.ctypes.data_as(_D))
    return b, (diag, sub)


# ----------------------------------------------------------------------------
# API
# ----------------------------------------------------------------------------

def release_cached_memory() -> None:
    """Return the library's idle cached device blocks to the driver
    (sts_release_cached_memory)."""
    load().sts_release_cached_memory()


def default_opts(**kw) -> Opts:
    o = Opts()
    load().sts_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def time_matrices(t):
    """(Dt diag, Dt sub, Mt diag, Mt sub) of the hat/indicator pair on nodes t."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    nt = len(t) - 1
    out = [np.empty(nt), np.empty(max(nt - 1, 1)), np.empty(nt), np.empty(max(nt - 1, 1))]
    _check(load().sts_time_matrices(nt, t.ctypes.data_as(_D), *[a.ctypes.data_as(_D) for a in out]))
    return out[0], out[1][: nt - 1], out[2], out[3][: nt - 1]


class Problem:
    """A space-time heat problem held by the library (sts_create / sts_destroy).

    F1 (Nh x P) and F2 (Nt x P) may be NumPy arrays (copied from host memory)
    or float64 CUDA tensors (copied on the device).  ``dt``/``mt`` are the
    (diag, sub) pairs of the lower-bidiagonal time matrices.
    """

    def __init__(self, dim: int, n: int, mu: float, dt, mt, F1, F2, stream=None):
        lib = load()
        self._lib = lib
        self.space = make_space(dim, n, mu)
        self._Dt, self._keep_dt = _bidiag(*dt)
        self._Mt, self._keep_mt = _bidiag(*mt)
        self.nt = len(self._keep_dt[0])
        self.device_inputs = _is_torch(F1)
        if self.device_inputs:
            self._stream = _stream_handle(stream)
            f1, p1, ld1 = dev_colmajor(F1)
            f2, p2, ld2 = dev_colmajor(F2)
            self._keep_f = (f1, f2)
            mem = STS_MEM_DEVICE
        else:
            self._stream = C.c_void_p(0) if stream is None else _stream_handle(stream)
            f1, f2 = _host_colmajor(F1), _host_colmajor(F2)
            p1, ld1 = C.c_void_p(f1.ctypes.data), f1.shape[0]
            p2, ld2 = C.c_void_p(f2.ctypes.data), f2.shape[0]
            self._keep_f = (f1, f2)
            mem = STS_MEM_HOST
        self.p = int(f1.shape[1])
        self.nh = int(f1.shape[0])
        h = C.c_void_p()
        _check(lib.sts_create(C.byref(self.space), C.byref(self._Dt), C.byref(self._Mt), self.nt,
                              self.p, p1, ld1, p2, ld2, mem, self._stream, C.byref(h)))
        self._h = h

    def solve(self, **opts) -> dict:
        o = default_opts(**opts)
        info = Info()
        code = self._lib.sts_solve(self._h, C.byref(o), C.byref(info))
        d = info.as_dict()
        d["status"] = STATUS_NAMES.get(code, code)
        # not converged, or a space that stopped growing above tol (breakdown):
        # the factors of the last iterate are kept and the info is returned
        if code not in (STS_OK, STS_E_NOT_CONVERGED) and not (code == STS_E_NUMERIC
                                                              and d["breakdown"] == 1):
            _check(code)
        d["error"] = self._lib.sts_last_error().decode() if code != STS_OK else ""
        return d

    def kernel_profile(self) -> dict:
        """{name: (seconds, launches, algorithmic bytes)} of the last profiled solve."""
        out = {}
        for k in range(STS_K_COUNT):
            sec, n, by = C.c_double(), C.c_int64(), C.c_double()
            _check(self._lib.sts_kernel_profile(self._h, k, C.byref(sec), C.byref(n), C.byref(by)))
            out[self._lib.sts_kernel_name(k).decode()] = (sec.value, n.value, by.value)
        return out

    def rank(self) -> int:
        k = C.c_int64()
        _check(self._lib.sts_rank(self._h, C.byref(k)))
        return int(k.value)

    def factors(self, device: bool = False):
        """(V, Y): NumPy arrays, or CUDA tensors if device=True."""
        k = self.rank()
        if device:
            V, Y = dev_empty(self.nh, k), dev_empty(k, self.nt)
            _check(self._lib.sts_get_factors(self._h, C.c_void_p(V.data_ptr()), max(self.nh, 1),
                                             C.c_void_p(Y.data_ptr()), max(k, 1), STS_MEM_DEVICE,
                                             self._stream))
            return V, Y
        V = np.zeros((self.nh, k), order="F")
        Y = np.zeros((k, self.nt), order="F")
        _check(self._lib.sts_get_factors(self._h, C.c_void_p(V.ctypes.data), max(self.nh, 1),
                                         C.c_void_p(Y.ctypes.data), max(k, 1), STS_MEM_HOST,
                                         self._stream))
        return V, Y

    def solution_columns(self, cols, device: bool = False):
        """U[:, cols] of U = V Y (time indices 0..nt-1), computed on the device
        without copying V; a NumPy array, or a CUDA tensor if device=True."""
        idx = (C.c_int64 * len(cols))(*[int(c) for c in cols])
        n = len(cols)
        if device:
            U = dev_empty(self.nh, n)
            _check(self._lib.sts_solution_columns(self._h, idx, n, C.c_void_p(U.data_ptr()),
                                                  max(self.nh, 1), STS_MEM_DEVICE, self._stream))
            return U
        U = np.zeros((self.nh, n), order="F")
        _check(self._lib.sts_solution_columns(self._h, idx, n, C.c_void_p(U.ctypes.data),
                                              max(self.nh, 1), STS_MEM_HOST, self._stream))
        return U

    def true_residual(self) -> float:
        r = C.c_double()
        _check(self._lib.sts_true_residual(self._h, C.byref(r)))
        return r.value

    def numerical_rank(self) -> int:
        r = C.c_int64()
        _check(self._lib.sts_numerical_rank(self._h, C.byref(r)))
        return int(r.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sts_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---- step-level calls (device tensors) ----

def apply_op(space: Space, op: int, X):
    X, px, ldx = dev_colmajor(X)
    Y = dev_empty(X.shape[0], X.shape[1])
    _check(load().sts_apply_op(C.byref(space), op, px, ldx, C.c_void_p(Y.data_ptr()),
                               max(Y.shape[0], 1), X.shape[1], _stream_handle()))
    return Y


def cg(space: Space, ops, B, rtol: float = 1e-12, maxit: int = 200000, check: bool = True):
    B, pb, ldb = dev_colmajor(B)
    X = dev_zeros(B.shape[0], B.shape[1])
    ops_a = (C.c_int32 * len(ops))(*ops)
    its = (C.c_int32 * len(ops))()
    code = load().sts_cg(C.byref(space), ops_a, pb, ldb, C.c_void_p(X.data_ptr()), X.shape[0],
                         B.shape[1], rtol, maxit, its, _stream_handle())
    if check:
        _check(code)
    return X, list(its), code


def pcg_mg(space: Space, B, rtol: float = 1e-12, maxit: int = 1000, check: bool = True):
    """Kx X = B by multigrid-preconditioned CG (2-D P1 and 3-D seven-point spaces whose n halves)."""
    B, pb, ldb = dev_colmajor(B)
    X = dev_zeros(B.shape[0], B.shape[1])
    its = (C.c_int32 * B.shape[1])()
    code = load().sts_pcg_mg(C.byref(space), pb, ldb, C.c_void_p(X.data_ptr()), X.shape[0],
                             B.shape[1], rtol, maxit, its, _stream_handle())
    if check:
        _check(code)
    return X, list(its), code


def pcg_mg_mixed(space: Space, B, shift: float = 0.0, rtol: float = 1e-12, maxit: int = 1000,
                 check: bool = True):
    """(Kx + shift Mx) X = B by FP64 CG preconditioned with the FP32-storage
    V-cycle (3-D seven-point spaces with a smoothed level)."""
    B, pb, ldb = dev_colmajor(B)
    X = dev_zeros(B.shape[0], B.shape[1])
    its = (C.c_int32 * B.shape[1])()
    code = load().sts_pcg_mg_mixed(C.byref(space), float(shift), pb, ldb,
                                   C.c_void_p(X.data_ptr()), X.shape[0], B.shape[1], rtol, maxit,
                                   its, _stream_handle())
    if check:
        _check(code)
    return X, list(its), code


def pcg_mg_refined(space: Space, B, rtol: float = 1e-12, maxit: int = 1000):
    """Kx X = B by FP32 multigrid PCG inside FP64 defect correction (3-D
    seven-point spaces with a smoothed level); returns (X, FP32 iterations,
    FP64 iterations, defect corrections)."""
    B, pb, ldb = dev_colmajor(B)
    X = dev_zeros(B.shape[0], B.shape[1])
    i32, i64, rounds = C.c_int64(), C.c_int64(), C.c_int64()
    _check(load().sts_pcg_mg_refined(C.byref(space), pb, ldb, C.c_void_p(X.data_ptr()), X.shape[0],
                                     B.shape[1], rtol, maxit, C.byref(i32), C.byref(i64),
                                     C.byref(rounds), _stream_handle()))
    return X, i32.value, i64.value, rounds.value


def mass_solve(space: Space, B, rtol: float = 1e-13):
    """Mx X = B: Chebyshev iteration (2-D P1) or direct line solves (3-D trilinear); returns (X, iterations)."""
    B, pb, ldb = dev_colmajor(B)
    X = dev_zeros(B.shape[0], B.shape[1])
    its = (C.c_int32 * B.shape[1])()
    _check(load().sts_mass_solve(C.byref(space), pb, ldb, C.c_void_p(X.data_ptr()), X.shape[0],
                                 B.shape[1], rtol, its, _stream_handle()))
    return X, its[0]


def tridiag_solve(space: Space, ops, B):
    """A X = B with A = Kx or Mx per column (ops), 1-D P1, direct."""
    B, pb, ldb = dev_colmajor(B)
    X = dev_empty(B.shape[0], B.shape[1])
    o = (C.c_int32 * B.shape[1])(*ops)
    _check(load().sts_tridiag_solve(C.byref(space), o, pb, ldb, C.c_void_p(X.data_ptr()),
                                    max(X.shape[0], 1), B.shape[1], _stream_handle()))
    return X


def adaptive_shift(ritz, shifts, a: float, b: float, grid: int = 1001) -> float:
    """Next rational Krylov shift (sts_adaptive_shift)."""
    r = np.ascontiguousarray(ritz, dtype=np.float64)
    sh = np.ascontiguousarray(shifts, dtype=np.float64)
    out = C.c_double()
    _check(load().sts_adaptive_shift(r.ctypes.data_as(_D) if len(r) else None, len(r),
                                     sh.ctypes.data_as(_D) if len(sh) else None, len(sh),
                                     float(a), float(b), int(grid), C.byref(out)))
    return out.value


def shifted_solve(space: Space, shift: float, B, rtol: float = 1e-13, maxit: int = 200000):
    """(Kx + shift Mx) X = B as the rational Krylov steps solve it; (X, iterations)."""
    B, pb, ldb = dev_colmajor(B)
    X = dev_empty(B.shape[0], B.shape[1])
    its = (C.c_int32 * B.shape[1])()
    _check(load().sts_shifted_solve(C.byref(space), float(shift), pb, ldb,
                                    C.c_void_p(X.data_ptr()), max(X.shape[0], 1), B.shape[1],
                                    rtol, maxit, its, _stream_handle()))
    return X, list(its)


def mg_vcycle(space: Space, R, shift: float = 0.0, fp32: bool = False):
    """Z = Bmg R, one multigrid V-cycle (the preconditioner of pcg_mg; with
    shift > 0 that of the shifted solves, for Kx + shift Mx); fp32 = the
    V-cycle with FP32 storage (sts_mg_vcycle_mixed)."""
    R, pr, ldr = dev_colmajor(R)
    Z = dev_empty(R.shape[0], R.shape[1])
    if fp32:
        _check(load().sts_mg_vcycle_mixed(C.byref(space), float(shift), pr, ldr,
                                          C.c_void_p(Z.data_ptr()), max(Z.shape[0], 1),
                                          R.shape[1], _stream_handle()))
    elif shift:
        _check(load().sts_mg_vcycle_shifted(C.byref(space), float(shift), pr, ldr,
                                            C.c_void_p(Z.data_ptr()), max(Z.shape[0], 1),
                                            R.shape[1], _stream_handle()))
    else:
        _check(load().sts_mg_vcycle(C.byref(space), pr, ldr, C.c_void_p(Z.data_ptr()),
                                    max(Z.shape[0], 1), R.shape[1], _stream_handle()))
    return Z


def m_orthonormalize(space: Space, V, MV, W, defl_tol: float = 1e-10):
    torch = _torch()
    W, pw, ldw = dev_colmajor(W.clone())
    MW = dev_empty(W.shape[0], W.shape[1])
    if V is None or V.shape[1] == 0:
        pv = pmv = C.c_void_p(0)
        ldv, k = max(W.shape[0], 1), 0
    else:
        V, pv, ldv = dev_colmajor(V)
        MV, pmv, ldmv = dev_colmajor(MV)
        assert ldmv == ldv
        k = V.shape[1]
    kept = C.c_int32()
    idx = (C.c_int32 * W.shape[1])()
    _check(load().sts_m_orthonormalize(C.byref(space), pv, pmv, ldv, k, pw,
                                       C.c_void_p(MW.data_ptr()), ldw, W.shape[1], defl_tol,
                                       C.byref(kept), idx, _stream_handle()))
    kv = kept.value
    return W[:, :kv], MW[:, :kv], [idx[j] for j in range(kv)]


def gram(A, B):
    A, pa, lda = dev_colmajor(A)
    B, pb, ldb = dev_colmajor(B)
    Cm = dev_empty(A.shape[1], B.shape[1])
    _check(load().sts_gram(A.shape[0], A.shape[1], B.shape[1], pa, lda, pb, ldb,
                           C.c_void_p(Cm.data_ptr()), A.shape[1], _stream_handle()))
    return Cm


def gram_noalloc(A, B, out=None):
    """C = A^T B through sts_gram_noalloc (no device allocation inside the
    call; `out`, an m x n column-major device tensor, receives C if given)."""
    A, pa, lda = dev_colmajor(A)
    B, pb, ldb = dev_colmajor(B)
    Cm = dev_empty(A.shape[1], B.shape[1]) if out is None else out
    _check(load().sts_gram_noalloc(A.shape[0], A.shape[1], B.shape[1], pa, lda, pb, ldb,
                                   C.c_void_p(Cm.data_ptr()), A.shape[1], _stream_handle()))
    return Cm


def dev_colmajor32(t):
    """A float32 CUDA tensor viewed as a column-major matrix -> (tensor, ptr, ld)."""
    torch = _torch()
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError("expected a float32 CUDA tensor")
    if t.dim() == 1:
        t = t[:, None]
    if t.stride(0) != 1 or (t.shape[1] > 1 and t.stride(1) < t.shape[0]):
        t = t.t().contiguous().t()
    ld = t.stride(1) if t.shape[1] > 1 else max(t.shape[0], 1)
    return t, C.c_void_p(t.data_ptr()), int(ld)


def gram_fp32(A32, B):
    """C = A32^T B in FP32 (A32 float32, B float64; C returned as float64)."""
    A32, pa, lda = dev_colmajor32(A32)
    B, pb, ldb = dev_colmajor(B)
    Cm = dev_empty(A32.shape[1], B.shape[1])
    _check(load().sts_gram_fp32(A32.shape[0], A32.shape[1], B.shape[1], pa, lda, pb, ldb,
                                C.c_void_p(Cm.data_ptr()), A32.shape[1], _stream_handle()))
    return Cm


def basis_update(A, Cm, W):
    A, pa, lda = dev_colmajor(A)
    Cm, pc, ldc = dev_colmajor(Cm)
    W, pw, ldw = dev_colmajor(W.clone())
    _check(load().sts_basis_update(A.shape[0], A.shape[1], W.shape[1], pa, lda, pc, ldc, pw, ldw,
                                   _stream_handle()))
    return W


def sym_eig(A):
    A, pa, lda = dev_colmajor(A)
    k = A.shape[0]
    lam = dev_empty(k, 1)
    Q = dev_empty(k, k)
    _check(load().sts_sym_eig(k, pa, lda, C.c_void_p(lam.data_ptr()), C.c_void_p(Q.data_ptr()), k,
                              _stream_handle()))
    return lam[:, 0], Q


def time_sweep(lam, Q, beta, F2, dt, mt):
    lam, pl, _ = dev_colmajor(lam)
    Q, pq, ldq = dev_colmajor(Q)
    beta, pb, ldb = dev_colmajor(beta)
    F2, pf, ldf = dev_colmajor(F2)
    k, nt, p = Q.shape[0], F2.shape[0], F2.shape[1]
    Dt, kd = _bidiag(*dt)
    Mt, km = _bidiag(*mt)
    Y = dev_empty(k, nt)
    _check(load().sts_time_sweep(k, nt, p, pl, pq, ldq, pb, ldb, pf, ldf, C.byref(Dt), C.byref(Mt),
                                 C.c_void_p(Y.data_ptr()), k, _stream_handle()))
    return Y


class Pool:
    """Solves many problems on one GPU, up to ``workers`` at a time
    (sts_pool_create / sts_pool_solve / sts_pool_destroy)."""

    def __init__(self, workers: int):
        self._lib = load()
        h = C.c_void_p()
        _check(self._lib.sts_pool_create(int(workers), C.byref(h)))
        self._h = h
        self.workers = int(workers)

    def solve(self, problems, opts=None, **common) -> list:
        """Solve every Problem in ``problems``; ``opts`` is one dict of
        options per problem (or None: ``common`` for all).  Returns one info
        dict per problem, with its "status" and "error"."""
        n = len(problems)
        handles = (C.c_void_p * max(n, 1))(*[pr._h for pr in problems])
        if opts is None:
            arr = (Opts * 1)(default_opts(**common))
            nopts = 1
        else:
            if len(opts) != n:
                raise ValueError("one options dict per problem")
            arr = (Opts * max(n, 1))(*[default_opts(**{**common, **o}) for o in opts])
            nopts = n
        infos = (Info * max(n, 1))()
        status = (C.c_int * max(n, 1))(*([-1] * max(n, 1)))
        code = self._lib.sts_pool_solve(self._h, n, handles, arr, nopts, infos, status)
        if code != STS_OK and any(status[i] == -1 for i in range(n)):
            _check(code)          # rejected before any solve started
        msg = self._lib.sts_last_error().decode() if code != STS_OK else ""
        out = []
        for i in range(n):
            d = infos[i].as_dict()
            d["status"] = STATUS_NAMES.get(status[i], status[i])
            d["error"] = ""
            out.append(d)
        if code != STS_OK:
            first = min(i for i in range(n) if status[i] != STS_OK)
            out[first]["error"] = msg
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sts_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def footprint(dim: int, n: int, nt: int, p: int, **opts) -> int:
    """Device bytes a problem of this shape holds once solved (sts_footprint)."""
    space = make_space(dim, n)
    return int(load().sts_footprint(C.byref(space), nt, p, C.byref(default_opts(**opts))))


class ServedProblem:
    """A finished request's problem, owned by the server until release."""

    def __init__(self, lib, handle, nh: int, nt: int):
        self._lib, self._h, self.nh, self.nt = lib, handle, nh, nt
        self._stream = C.c_void_p(0)

    rank = Problem.rank
    factors = Problem.factors
    true_residual = Problem.true_residual
    numerical_rank = Problem.numerical_rank


class Server:
    """Request queue in front of the solver (sts_server_*)."""

    def __init__(self, workers: int, mem_budget: int):
        self._lib = load()
        h = C.c_void_p()
        _check(self._lib.sts_server_create(int(workers), int(mem_budget), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, dim: int, n: int, mu: float, dt, mt, F1, F2, **opts) -> int:
        """Queue one problem (host arrays); returns its ticket."""
        dd, ds = (np.ascontiguousarray(a, dtype=np.float64) for a in dt)
        md, ms = (np.ascontiguousarray(a, dtype=np.float64) for a in mt)
        f1, f2 = _host_colmajor(F1), _host_colmajor(F2)
        r = Request()
        r.space = make_space(dim, n, mu)
        r.nt = len(dd)
        r.p = f1.shape[1]
        ds = ds if len(ds) else np.zeros(1)
        ms = ms if len(ms) else np.zeros(1)
        r.dt_diag, r.dt_sub = dd.ctypes.data_as(_D), ds.ctypes.data_as(_D)
        r.mt_diag, r.mt_sub = md.ctypes.data_as(_D), ms.ctypes.data_as(_D)
        r.F1, r.ldf1 = f1.ctypes.data_as(_D), f1.shape[0]
        r.F2, r.ldf2 = f2.ctypes.data_as(_D), f2.shape[0]
        r.opts = default_opts(**opts)
        t = C.c_int64()
        _check(self._lib.sts_server_submit(self._h, C.byref(r), C.byref(t)))
        self._keep[t.value] = (int(np.prod([r.space.n[d] for d in range(3)])), r.nt)
        return int(t.value)

    def wait(self, ticket: int, timeout: float = -1.0):
        """(result dict, ServedProblem or None) once the request has finished."""
        res = Result()
        h = C.c_void_p()
        _check(self._lib.sts_server_wait(self._h, int(ticket), float(timeout), C.byref(res),
                                         C.byref(h)))
        d = res.info.as_dict()
        d.update(status=STATUS_NAMES.get(res.status, res.status),
                 queued_seconds=res.queued_seconds, latency_seconds=res.latency_seconds,
                 footprint=res.footprint,
                 error=self._lib.sts_last_error().decode() if res.status != STS_OK else "")
        nh, nt = self._keep[int(ticket)]
        return d, (ServedProblem(self._lib, h, nh, nt) if h.value else None)

    def release(self, ticket: int):
        _check(self._lib.sts_server_release(self._h, int(ticket)))
        self._keep.pop(int(ticket), None)

    def stats(self) -> dict:
        st = ServerStats()
        _check(self._lib.sts_server_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sts_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
