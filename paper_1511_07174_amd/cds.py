"""Thin Python binding of libcds.so (the C-ABI in include/cds.h).

Argument marshalling only: every step of a factorization or solve runs in the
HIP kernels of the library.  PyTorch provides the device memory (tensors and
the workspace) and the stream (torch's current stream).  If the library is
missing the binding raises; there is no CPU fallback.

Matrices are column-major: a (n, m) tensor with strides (1, ld), e.g.
``colmajor(t)``; batches are (batch, n, m) with strides (s, 1, ld).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcds.so")

SUCCESS = 0
OP_N, OP_T = 0, 1
LOWER = 0
R_64F, R_32F = 0, 1
PREC = {"fp32": 0, "bf16": 1, "fp16": 2}
OPT_NB, OPT_LOOKAHEAD, OPT_LEAF, OPT_PANEL_WGS, OPT_KERNEL_TIMING = 0, 1, 2, 3, 4
KC = {"update": 0, "panel": 1, "laswp": 2, "trsm": 3, "trsv": 4, "residual": 5, "krylov_gemv": 6}
TUNE_GETRF_NB, TUNE_POTRF_NB, TUNE_VBATCH_TILE = 0, 1, 2


class CdsError(RuntimeError):
    pass


class IrParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("success_tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("host_check", ctypes.c_int32), ("reserved", ctypes.c_int32)]


IR_RESULT_BYTES = 40   # int32 iters, info, converged, fell_back; double eta, eta0; int32 stop_reason, reserved

KRYLOV = {"cg": 0, "bicg": 1, "bicgstab": 2, "gmres": 3}


class KrylovParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("reserved", ctypes.c_int32)]


KRYLOV_RESULT_BYTES = 24   # int32 iters, converged, breakdown, reserved; double relres


def krylov_params(**kw) -> KrylovParams:
    p = KrylovParams(1e-10, 1000, 30, 10, 0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p

_lib = None


def lib():
    """Load libcds.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CdsError("libcds.so not found at %s: build it first (paper_1511_07174_amd/build.py)" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    P, I64, I32, D, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    PSZ = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "cds_create": [ctypes.POINTER(P)],
        "cds_destroy": [P],
        "cds_set_stream": [P, P],
        "cds_get_stream": [P, ctypes.POINTER(P)],
        "cds_set_workspace": [P, P, SZ],
        "cds_set_option": [P, ctypes.c_int, I64],
        "cds_tune_set": [P, ctypes.c_int, ctypes.c_int, I64, I64],
        "cds_tune_clear": [P],
        "cds_tune": [P, ctypes.c_char_p],
        "cds_tune_check": [ctypes.c_char_p, ctypes.POINTER(I64)],
        "cds_device_error": [P, ctypes.POINTER(I32)],
        "cds_getrf_bufferSize": [P, ctypes.c_int, I64, I64, PSZ],
        "cds_getrs_bufferSize": [P, ctypes.c_int, I64, I64, I64, PSZ],
        "cds_potrf_bufferSize": [P, ctypes.c_int, I64, PSZ],
        "cds_potrs_bufferSize": [P, ctypes.c_int, I64, I64, PSZ],
        "cds_gesv_mixed_bufferSize": [P, ctypes.c_int, I64, I64, I64, P, PSZ],
        "cds_posv_mixed_bufferSize": [P, ctypes.c_int, I64, I64, P, PSZ],
        "cds_posv_mixed_vbatched_bufferSize": [P, I64, I64, I64, PSZ],
        "cds_dgetrf": [P, I64, P, I64, P, P],
        "cds_sgetrf": [P, I64, P, I64, P, P],
        "cds_dgetrf_strided_batched": [P, I64, P, I64, I64, P, I64, P, I64],
        "cds_sgetrf_strided_batched": [P, I64, P, I64, I64, P, I64, P, I64],
        "cds_dgetrs": [P, ctypes.c_int, I64, I64, P, I64, P, P, I64],
        "cds_sgetrs": [P, ctypes.c_int, I64, I64, P, I64, P, P, I64],
        "cds_dgetrs_strided_batched": [P, ctypes.c_int, I64, I64, P, I64, I64, P, I64, P, I64, I64, I64],
        "cds_dpotrf": [P, ctypes.c_int, I64, P, I64, P],
        "cds_spotrf": [P, ctypes.c_int, I64, P, I64, P],
        "cds_dpotrs": [P, ctypes.c_int, I64, I64, P, I64, P, I64],
        "cds_spotrs": [P, ctypes.c_int, I64, I64, P, I64, P, I64],
        "cds_dgesv_mixed": [P, ctypes.c_int, I64, I64, P, I64, P, I64, P, I64, P, P, P, P],
        "cds_dgesv_mixed_noalloc": [P, ctypes.c_int, I64, I64, P, I64, P, I64, P, I64, P, P, P, P],
        "cds_dgesv_mixed_strided_batched": [P, ctypes.c_int, I64, I64, P, I64, I64, P, I64, I64, P, I64, I64, P, I64,
                                            P, I64, P, P, I64],
        "cds_dgetrs_mixed_strided_batched": [P, ctypes.c_int, I64, I64, P, I64, I64, P, I64, P, I64, P, I64, I64, P,
                                             I64, I64, P, P, I64],
        "cds_dposv_mixed": [P, ctypes.c_int, ctypes.c_int, I64, I64, P, I64, P, I64, P, I64, P, P, P],
        "cds_dposv_mixed_vbatched": [P, ctypes.c_int, I64, I64, P, P, P, P, P, P, P, I64, P, P, P, P, P],
        "cds_krylov_bufferSize": [P, ctypes.c_int, I64, I32, PSZ],
        "cds_dkrylov": [P, ctypes.c_int, I64, P, I64, P, P, P, P],
        "cds_gesv_gmres_ir_bufferSize": [P, ctypes.c_int, I64, I32, PSZ],
        "cds_dgesv_gmres_ir": [P, ctypes.c_int, I64, P, I64, P, P, P, P, P, P, P],
        "cds_douter_strided_batched": [P, I64, I64, I64, D, P, I64, I64, P, I64, I64, P, I64, I64, I64],
        "cds_kernel_timing": [P, I32, ctypes.POINTER(I64), ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)],
        "cds_kernel_timing_reset": [P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.cds_status_string.argtypes = [ctypes.c_int]
    L.cds_status_string.restype = ctypes.c_char_p


EXPORTED = [
    "cds_create", "cds_destroy", "cds_set_stream", "cds_get_stream", "cds_set_workspace", "cds_set_option",
    "cds_tune_set", "cds_tune_clear", "cds_tune", "cds_tune_check", "cds_device_error", "cds_status_string",
    "cds_getrf_bufferSize", "cds_getrs_bufferSize", "cds_potrf_bufferSize", "cds_potrs_bufferSize",
    "cds_gesv_mixed_bufferSize", "cds_posv_mixed_bufferSize", "cds_posv_mixed_vbatched_bufferSize",
    "cds_dgetrf", "cds_sgetrf", "cds_dgetrf_strided_batched", "cds_sgetrf_strided_batched",
    "cds_dgetrs", "cds_sgetrs", "cds_dgetrs_strided_batched",
    "cds_dpotrf", "cds_spotrf", "cds_dpotrs", "cds_spotrs",
    "cds_dgesv_mixed", "cds_dgesv_mixed_noalloc", "cds_dgesv_mixed_strided_batched", "cds_dgetrs_mixed_strided_batched",
    "cds_dposv_mixed", "cds_dposv_mixed_vbatched", "cds_douter_strided_batched",
    "cds_krylov_bufferSize", "cds_dkrylov", "cds_gesv_gmres_ir_bufferSize", "cds_dgesv_gmres_ir",
    "cds_kernel_timing", "cds_kernel_timing_reset",
]


def check(status: int, what: str = ""):
    if status != SUCCESS:
        msg = lib().cds_status_string(status).decode()
        raise CdsError("%s failed: %s (%d)" % (what, msg, status))


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def colmajor(t: torch.Tensor) -> torch.Tensor:
    """Column-major copy of a matrix (..., n, m): strides (..., 1, n).  Always a new
    tensor, so that the functional API never writes into its arguments."""
    return t.transpose(-1, -2).clone(memory_format=torch.contiguous_format).transpose(-1, -2)


def _ld(t: torch.Tensor) -> int:
    if t.dim() == 1:
        return max(1, t.shape[0])
    if t.stride(-2) != 1 and t.shape[-2] > 1:
        raise CdsError("matrix must be column-major (stride 1 along rows), got strides %s" % (t.stride(),))
    return max(1, t.stride(-1) if t.shape[-1] > 1 else t.shape[-2])


def _bstride(t: torch.Tensor) -> int:
    return t.stride(0) if t.dim() == 3 else 0


@dataclass
class KrylovResult:
    iters: int
    converged: bool
    breakdown: bool
    relres: float


def decode_krylov(buf: torch.Tensor) -> KrylovResult:
    h = buf.cpu()
    ints = h[:16].view(torch.int32).tolist()
    return KrylovResult(ints[0], bool(ints[1]), bool(ints[2]), h[16:24].view(torch.float64).tolist()[0])


@dataclass
class IrResult:
    iters: int
    info: int
    converged: bool
    fell_back: bool
    eta: float
    eta0: float
    stop_reason: int


def decode_results(buf: torch.Tensor):
    """Decode a uint8 device buffer of cds_ir_result_t records (copies to host)."""
    h = buf.cpu()
    n = h.numel() // IR_RESULT_BYTES
    out = []
    for i in range(n):
        rec = h[i * IR_RESULT_BYTES:(i + 1) * IR_RESULT_BYTES]
        ints = rec[:16].view(torch.int32).tolist()
        dbl = rec[16:32].view(torch.float64).tolist()
        tail = rec[32:40].view(torch.int32).tolist()
        out.append(IrResult(ints[0], ints[1], bool(ints[2]), bool(ints[3]), dbl[0], dbl[1], tail[0]))
    return out


class Handle:
    """A cds handle bound to the current device, with a torch-allocated workspace."""

    def __init__(self):
        h = ctypes.c_void_p()
        check(lib().cds_create(ctypes.byref(h)), "cds_create")
        self.h = h
        self._ws = None
        self._ws_bytes = 0

    def close(self):
        if self.h:
            lib().cds_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- plumbing
    def bind(self, need_bytes: int, device=None):
        """Bind torch's current stream and make the workspace at least need_bytes."""
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        stream = torch.cuda.current_stream(dev)
        check(lib().cds_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), "cds_set_stream")
        need = max(int(need_bytes), 256)
        if self._ws is None or self._ws_bytes < need:
            self._ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
            base = self._ws.data_ptr()
            aligned = (base + 255) // 256 * 256
            self._ws_ptr = aligned
            self._ws_bytes = need
            check(lib().cds_set_workspace(self.h, ctypes.c_void_p(aligned), ctypes.c_size_t(need)), "cds_set_workspace")

    def set_option(self, opt: int, value: int):
        check(lib().cds_set_option(self.h, opt, value), "cds_set_option")

    def tune_set(self, key: int, dtype: int, n_max: int, value: int):
        check(lib().cds_tune_set(self.h, key, dtype, n_max, value), "cds_tune_set")

    def tune_clear(self):
        check(lib().cds_tune_clear(self.h), "cds_tune_clear")

    def tune(self, path: str):
        """Install the autotuner's JSON table (parsed by the library, cds_tune)."""
        check(lib().cds_tune(self.h, os.fsencode(path)), "cds_tune")

    def kernel_timing(self, kc: str):
        """(launches, ms, flops, bytes) summed over the recorded launches of a kernel class."""
        n = ctypes.c_int64(0)
        ms, fl, by = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        check(lib().cds_kernel_timing(self.h, KC[kc], ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl),
                                      ctypes.byref(by)), "cds_kernel_timing")
        return n.value, ms.value, fl.value, by.value

    def kernel_timing_reset(self):
        check(lib().cds_kernel_timing_reset(self.h), "cds_kernel_timing_reset")

    def device_error(self) -> int:
        v = ctypes.c_int32(0)
        check(lib().cds_device_error(self.h, ctypes.byref(v)), "cds_device_error")
        return v.value

    def _size(self, fn, *args) -> int:
        out = ctypes.c_size_t(0)
        check(getattr(lib(), fn)(self.h, *args, ctypes.byref(out)), fn)
        return out.value

    # -- LU
    def getrf_(self, A: torch.Tensor, ipiv: torch.Tensor, info: torch.Tensor):
        """In-place LU of a column-major matrix or a strided batch of them."""
        batched = A.dim() == 3
        n = A.shape[-1]
        dt = R_64F if A.dtype == torch.float64 else R_32F
        batch = A.shape[0] if batched else 1
        self.bind(self._size("cds_getrf_bufferSize", dt, n, batch), A.device)
        if not batched:
            fn = lib().cds_dgetrf if dt == R_64F else lib().cds_sgetrf
            check(fn(self.h, n, _p(A), _ld(A), _p(ipiv), _p(info)), "getrf")
        else:
            fn = lib().cds_dgetrf_strided_batched if dt == R_64F else lib().cds_sgetrf_strided_batched
            check(fn(self.h, n, _p(A), _ld(A), _bstride(A), _p(ipiv), ipiv.stride(0), _p(info), batch), "getrf_batched")

    def getrs_(self, LU: torch.Tensor, ipiv: torch.Tensor, B: torch.Tensor, trans: bool = False):
        batched = LU.dim() == 3
        n = LU.shape[-1]
        nrhs = B.shape[-1] if B.dim() == LU.dim() else 1
        dt = R_64F if LU.dtype == torch.float64 else R_32F
        batch = LU.shape[0] if batched else 1
        self.bind(self._size("cds_getrs_bufferSize", dt, n, nrhs, batch), LU.device)
        op = OP_T if trans else OP_N
        ldb = _ld(B) if B.dim() == LU.dim() else n
        if not batched:
            fn = lib().cds_dgetrs if dt == R_64F else lib().cds_sgetrs
            check(fn(self.h, op, n, nrhs, _p(LU), _ld(LU), _p(ipiv), _p(B), ldb), "getrs")
        else:
            if dt != R_64F:
                raise CdsError("batched getrs is FP64")
            check(lib().cds_dgetrs_strided_batched(self.h, op, n, nrhs, _p(LU), _ld(LU), _bstride(LU), _p(ipiv),
                                                   ipiv.stride(0), _p(B), ldb, B.stride(0), batch), "getrs_batched")

    # -- Cholesky
    def potrf_(self, A: torch.Tensor, info: torch.Tensor):
        n = A.shape[-1]
        dt = R_64F if A.dtype == torch.float64 else R_32F
        self.bind(self._size("cds_potrf_bufferSize", dt, n), A.device)
        fn = lib().cds_dpotrf if dt == R_64F else lib().cds_spotrf
        check(fn(self.h, LOWER, n, _p(A), _ld(A), _p(info)), "potrf")

    def potrs_(self, L: torch.Tensor, B: torch.Tensor):
        n = L.shape[-1]
        nrhs = B.shape[-1] if B.dim() == 2 else 1
        dt = R_64F if L.dtype == torch.float64 else R_32F
        self.bind(self._size("cds_potrs_bufferSize", dt, n, nrhs), L.device)
        fn = lib().cds_dpotrs if dt == R_64F else lib().cds_spotrs
        check(fn(self.h, LOWER, n, nrhs, _p(L), _ld(L), _p(B), _ld(B) if B.dim() == 2 else n), "potrs")

    # -- mixed precision
    def gesv_mixed(self, A, B, X, LUlo, ipiv, results, precision="fp32", params: IrParams | None = None):
        batched = A.dim() == 3
        n = A.shape[-1]
        nrhs = B.shape[-1] if B.dim() == A.dim() else 1
        batch = A.shape[0] if batched else 1
        prm = params or default_params()
        self.bind(self._size("cds_gesv_mixed_bufferSize", PREC[precision], n, nrhs, batch,
                             ctypes.byref(prm)), A.device)
        ldb = _ld(B) if B.dim() == A.dim() else n
        ldx = _ld(X) if X.dim() == A.dim() else n
        check(lib().cds_dgesv_mixed_strided_batched(
            self.h, PREC[precision], n, nrhs, _p(A), _ld(A), _bstride(A), _p(B), ldb, _bstride(B), _p(X), ldx,
            _bstride(X), _p(LUlo), LUlo.stride(0) if batched else n * n, _p(ipiv), ipiv.stride(0) if batched else n,
            ctypes.byref(prm), _p(results), batch), "gesv_mixed")

    def gesv_mixed_noalloc(self, A, B, X, LUlo, ipiv, result, precision="fp32", params: IrParams | None = None):
        """cds_dgesv_mixed_noalloc: one system, the library's fixed scratch instead of a workspace
        (binds torch's current stream only)."""
        n = A.shape[-1]
        nrhs = B.shape[-1] if B.dim() == 2 else 1
        prm = params or default_params()
        stream = torch.cuda.current_stream(A.device)
        check(lib().cds_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), "cds_set_stream")
        ldb = _ld(B) if B.dim() == 2 else n
        ldx = _ld(X) if X.dim() == 2 else n
        check(lib().cds_dgesv_mixed_noalloc(self.h, PREC[precision], n, nrhs, _p(A), _ld(A), _p(B), ldb, _p(X), ldx,
                                            _p(LUlo), _p(ipiv), ctypes.byref(prm), _p(result)), "gesv_mixed_noalloc")

    def getrs_mixed(self, A, LUlo, ipiv, B, X, results, trans=False, params: IrParams | None = None):
        batched = A.dim() == 3
        n = A.shape[-1]
        nrhs = B.shape[-1] if B.dim() == A.dim() else 1
        batch = A.shape[0] if batched else 1
        prm = params or default_params()
        self.bind(self._size("cds_gesv_mixed_bufferSize", 0, n, nrhs, batch, ctypes.byref(prm)), A.device)
        ldb = _ld(B) if B.dim() == A.dim() else n
        ldx = _ld(X) if X.dim() == A.dim() else n
        check(lib().cds_dgetrs_mixed_strided_batched(
            self.h, OP_T if trans else OP_N, n, nrhs, _p(A), _ld(A), _bstride(A), _p(LUlo),
            LUlo.stride(0) if batched else n * n, _p(ipiv), ipiv.stride(0) if batched else n, _p(B), ldb,
            _bstride(B), _p(X), ldx, _bstride(X), ctypes.byref(prm), _p(results), batch), "getrs_mixed")

    def posv_mixed(self, A, B, X, Llo, result, precision="fp32", params: IrParams | None = None):
        n = A.shape[-1]
        nrhs = B.shape[-1] if B.dim() == 2 else 1
        prm = params or default_params()
        self.bind(self._size("cds_posv_mixed_bufferSize", PREC[precision], n, nrhs, ctypes.byref(prm)), A.device)
        check(lib().cds_dposv_mixed(self.h, PREC[precision], LOWER, n, nrhs, _p(A), _ld(A), _p(B),
                                    _ld(B) if B.dim() == 2 else n, _p(X), _ld(X) if X.dim() == 2 else n, _p(Llo),
                                    ctypes.byref(prm), _p(result)), "posv_mixed")

    def posv_mixed_vbatched(self, batch, nmax, n_dev, A_ptrs, lda, B_ptrs, ldb, X_ptrs, ldx, nrhs, results,
                            order=None, t_start=None, t_end=None, params: IrParams | None = None, device=None):
        prm = params or default_params()
        self.bind(self._size("cds_posv_mixed_vbatched_bufferSize", batch, nmax, nrhs), device)
        check(lib().cds_dposv_mixed_vbatched(self.h, PREC["fp32"], batch, nmax, _p(n_dev), _p(A_ptrs), _p(lda),
                                             _p(B_ptrs), _p(ldb), _p(X_ptrs), _p(ldx), nrhs, _p(order),
                                             ctypes.byref(prm), _p(results), _p(t_start), _p(t_end)),
              "posv_mixed_vbatched")

    # -- Krylov solvers
    def krylov(self, method: str, A, b, x, result, params: KrylovParams | None = None):
        """cds_dkrylov: x (initial guess in, solution out)."""
        n = A.shape[-1]
        prm = params or krylov_params()
        self.bind(self._size("cds_krylov_bufferSize", KRYLOV[method], n, prm.restart), A.device)
        check(lib().cds_dkrylov(self.h, KRYLOV[method], n, _p(A), _ld(A), _p(b), _p(x), ctypes.byref(prm),
                                _p(result)), "krylov_" + method)

    def gesv_gmres_ir(self, A, b, x, LUlo, ipiv, result, precision="bf16", params: IrParams | None = None,
                      inner: KrylovParams | None = None):
        n = A.shape[-1]
        prm = params or default_params()
        kp = inner or krylov_params(tol=1e-4, max_iter=60)
        self.bind(self._size("cds_gesv_gmres_ir_bufferSize", PREC[precision], n, kp.restart), A.device)
        check(lib().cds_dgesv_gmres_ir(self.h, PREC[precision], n, _p(A), _ld(A), _p(b), _p(x), _p(LUlo), _p(ipiv),
                                       ctypes.byref(prm), ctypes.byref(kp), _p(result)), "gesv_gmres_ir")

    def outer(self, X, Y, C, alpha=-1.0):
        """C = alpha X Y^T (strided batches when 3-D)."""
        batched = C.dim() == 3
        m, n = C.shape[-2], C.shape[-1]
        k = X.shape[-1] if X.dim() == C.dim() else 1
        batch = C.shape[0] if batched else 1
        ldx = _ld(X) if X.dim() == C.dim() else m
        ldy = _ld(Y) if Y.dim() == C.dim() else n
        stream = torch.cuda.current_stream(C.device)
        check(lib().cds_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)), "cds_set_stream")
        check(lib().cds_douter_strided_batched(self.h, m, n, k, float(alpha), _p(X), ldx,
                                               X.stride(0) if batched else 0, _p(Y), ldy,
                                               Y.stride(0) if batched else 0, _p(C), _ld(C),
                                               C.stride(0) if batched else 0, batch), "outer")


def default_params(**kw) -> IrParams:
    p = IrParams(1e-15, 1e-14, 30, 0, 0, 0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


_default_handle = None


def handle() -> Handle:
    """The package's handle; on creation it installs the tuning table (see tune.py)."""
    global _default_handle
    if _default_handle is None:
        _default_handle = Handle()
        from . import tune
        path = tune.default_table_path()
        if path.lower() != "none" and os.path.exists(path):
            _default_handle.tune(path)
    return _default_handle
