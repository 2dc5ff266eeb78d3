"""Plain CPU FP64 oracle for the direct solvers of arXiv 1511.07174 (Sec. 2).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the test suite, the smoke check and the benchmark's CPU-baseline leg may.
It shares no code with the HIP library; the two meet only through the seeded
input generators in ``synth``.

The arithmetic lives in ``oracle.c`` (plain C, FP64, no FMA contraction):
unblocked Gaussian elimination with partial pivoting, unblocked Cholesky,
substitutions, and a double-double residual.  This module wraps it with numpy
and adds the derived quantities the tests use:

* backward error  eta_inf = max_c ||b_c - A x_c||_inf / (||A||_inf ||x_c||_inf)
  (the paper defines no accuracy metric; this normwise form is the reading
  adopted for every check);
* reconstruction ratio rho = ||P A - L U||_inf / (n eps ||A||_inf);
* the adjoint of x = A^{-1} b: bbar = A^{-T} xbar, Abar = -bbar x^T;
* the closed-form solve for A = H1 diag(sigma) H2 built from Householder
  reflectors.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

EPS = 2.0 ** -52   # unit roundoff convention used for rho and eta/eps: 2^-52


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2 -fopenmp -ffp-contract=off)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        L.oracle_dgetrf.restype = I64
        L.oracle_dgetrf.argtypes = [I64, P, I64, P]
        L.oracle_sgetrf.restype = I64
        L.oracle_sgetrf.argtypes = [I64, P, I64, P]
        L.oracle_dgetrs.restype = None
        L.oracle_dgetrs.argtypes = [ctypes.c_int, I64, I64, P, I64, P, P, I64]
        L.oracle_dpotrf.restype = I64
        L.oracle_dpotrf.argtypes = [I64, P, I64]
        L.oracle_dpotrs.restype = None
        L.oracle_dpotrs.argtypes = [I64, I64, P, I64, P, I64]
        L.oracle_residual_dd.restype = None
        L.oracle_residual_dd.argtypes = [ctypes.c_int, I64, I64, P, I64, P, I64, P, I64, P, I64]
        L.oracle_norm_inf.restype = ctypes.c_double
        L.oracle_norm_inf.argtypes = [I64, I64, P, I64]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def _f64(a):
    return np.array(a, dtype=np.float64, order="F", copy=True)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _as2d(b):
    b = np.asarray(b, dtype=np.float64)
    return b.reshape(-1, 1) if b.ndim == 1 else b


# --------------------------------------------------------------------------------------
# factorizations and solves (Sec. 2: A = LU with partial pivoting or A = L L^T; Ly=b, Ux=y)
# --------------------------------------------------------------------------------------
def getrf(A):
    """GEPP of a square matrix: returns (LU, ipiv (1-based int32), info)."""
    LU = _f64(A)
    n = LU.shape[0]
    assert LU.shape == (n, n)
    ipiv = np.zeros(n, dtype=np.int32)
    info = lib().oracle_dgetrf(n, _ptr(LU), max(1, n), _ptr(ipiv))
    return LU, ipiv, int(info)


def sgetrf(A):
    """GEPP carried out entirely in FP32 (A is rounded to FP32 first): returns (LU float32, ipiv, info)."""
    LU = np.array(A, dtype=np.float32, order="F", copy=True)
    n = LU.shape[0]
    assert LU.shape == (n, n)
    ipiv = np.zeros(n, dtype=np.int32)
    info = lib().oracle_sgetrf(n, _ptr(LU), max(1, n), _ptr(ipiv))
    return LU, ipiv, int(info)


def getrs(LU, ipiv, B, trans: bool = False):
    """Solve A X = B (or A^T X = B) from getrf's factors; returns X with B's shape."""
    LU = _f64(LU)
    shape = np.shape(B)
    X = _f64(_as2d(B))
    n, nrhs = X.shape
    ip = np.ascontiguousarray(ipiv, dtype=np.int32)
    lib().oracle_dgetrs(1 if trans else 0, n, nrhs, _ptr(LU), max(1, n), _ptr(ip), _ptr(X), max(1, n))
    return X.reshape(shape)


def potrf(A):
    """Lower Cholesky; returns (L, info).  The strict upper triangle is returned unchanged."""
    L = _f64(A)
    n = L.shape[0]
    info = lib().oracle_dpotrf(n, _ptr(L), max(1, n))
    return L, int(info)


def potrs(L, B):
    L = _f64(L)
    shape = np.shape(B)
    X = _f64(_as2d(B))
    n, nrhs = X.shape
    lib().oracle_dpotrs(n, nrhs, _ptr(L), max(1, n), _ptr(X), max(1, n))
    return X.reshape(shape)


def residual_dd(A, X, B, trans: bool = False):
    """R = B - op(A) X accumulated in double-double, rounded once to FP64."""
    A = _f64(A)
    shape = np.shape(B)
    X2 = _f64(_as2d(X))
    B2 = _f64(_as2d(B))
    n, nrhs = B2.shape
    R = np.zeros((n, nrhs), dtype=np.float64, order="F")
    lib().oracle_residual_dd(1 if trans else 0, n, nrhs, _ptr(A), max(1, n), _ptr(X2), max(1, n),
                             _ptr(B2), max(1, n), _ptr(R), max(1, n))
    return R.reshape(shape)


def norm_inf(A):
    A = _f64(_as2d(A))
    return float(lib().oracle_norm_inf(A.shape[0], A.shape[1], _ptr(A), max(1, A.shape[0])))


def eta_inf(A, X, B, trans: bool = False):
    """Normwise backward error, maximised over right-hand-side columns."""
    R = _as2d(residual_dd(A, X, B, trans))
    X2 = _as2d(X)
    nA = norm_inf(np.asarray(A).T if trans else A)
    worst = 0.0
    for c in range(R.shape[1]):
        den = nA * np.max(np.abs(X2[:, c]))
        val = np.max(np.abs(R[:, c])) / den if den > 0 else (0.0 if not np.any(R[:, c]) else np.inf)
        if not np.isfinite(val):
            return float("inf")
        worst = max(worst, val)
    return float(worst)


# --------------------------------------------------------------------------------------
# derived checks
# --------------------------------------------------------------------------------------
def ipiv_to_perm(ipiv):
    """Row order p such that (P A) = A[p, :], from sequential interchanges."""
    n = len(ipiv)
    p = np.arange(n)
    for k in range(n):
        j = int(ipiv[k]) - 1
        p[k], p[j] = p[j], p[k]
    return p


def first_pivot_mismatch(ipiv_test, LU_ref, ipiv_ref):
    """Compare a pivot sequence with the oracle's.  Returns (k, mult): k = the first step whose pivot
    differs (len(ipiv) when none does) and mult = |l| of the row the tested sequence chose at step k,
    read from the oracle's own factor L.  Up to step k both sequences interchanged the same rows, so
    that row's multiplier in the oracle's elimination is |a(chosen, k)| / |a(pivot, k)| <= 1, and a
    value within rounding of 1 means the two rows tied for the pivot (a legitimate difference)."""
    a = np.asarray(ipiv_test).astype(np.int64) - 1
    b = np.asarray(ipiv_ref).astype(np.int64) - 1
    n = len(b)
    diff = np.nonzero(a != b)[0]
    if len(diff) == 0:
        return n, 1.0
    k = int(diff[0])
    pos = int(a[k])
    # the oracle's interchange at step k, then every later one, moves that row
    if pos == k:
        pos = int(b[k])
    for j in range(k + 1, n):
        q = int(b[j])
        if pos == j:
            pos = q
        elif pos == q:
            pos = j
    return k, float(abs(np.asarray(LU_ref)[pos, k]))


def unpack_lu(LU):
    LU = np.asarray(LU, dtype=np.float64)
    L = np.tril(LU, -1) + np.eye(LU.shape[0])
    U = np.triu(LU)
    return L, U


def rho_lu(A, LU, ipiv, eps: float = EPS):
    """||P A - L U||_inf / (n eps ||A||_inf)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    L, U = unpack_lu(LU)
    D = A[ipiv_to_perm(ipiv), :] - L @ U
    nA = norm_inf(A)
    return float(norm_inf(D) / (n * eps * nA)) if nA > 0 else float(norm_inf(D))


def rho_llt(A, L, eps: float = EPS):
    """||A - L L^T||_inf / (n eps ||A||_inf) using the lower triangle of A (A symmetric)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Ls = np.tril(np.asarray(L, dtype=np.float64))
    Asym = np.tril(A) + np.tril(A, -1).T
    D = Asym - Ls @ Ls.T
    return float(norm_inf(D) / (n * eps * norm_inf(Asym)))


def freivalds_lu(A, LU, ipiv, nprobe: int = 8, seed: int = 0):
    """max_v ||P A v - L (U v)||_inf / (||A||_inf ||v||_inf) over random probes; O(n^2) each."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    p = ipiv_to_perm(ipiv)
    LU = np.asarray(LU, dtype=np.float64)
    nA = norm_inf(A)
    worst = 0.0
    for _ in range(nprobe):
        v = rng.uniform(-1.0, 1.0, n)
        uv = np.triu(LU) @ v
        luv = np.tril(LU, -1) @ uv + uv
        pav = (A @ v)[p]
        worst = max(worst, float(np.max(np.abs(pav - luv)) / (nA * np.max(np.abs(v)))))
    return worst


def freivalds_llt(A, L, nprobe: int = 8, seed: int = 0):
    """max_v ||A v - L (L^T v)||_inf / (||A||_inf ||v||_inf) over random probes, with A read from its lower
    triangle (symmetric); O(n^2) per probe."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = np.tril(np.asarray(L, dtype=np.float64))
    Al = np.tril(A)
    nA = None
    worst = 0.0
    for _ in range(nprobe):
        v = rng.uniform(-1.0, 1.0, n)
        av = Al @ v + np.tril(A, -1).T @ v
        llv = Ls @ (Ls.T @ v)
        if nA is None:
            nA = norm_inf(Al + np.tril(A, -1).T)
        worst = max(worst, float(np.max(np.abs(av - llv)) / (nA * np.max(np.abs(v)))))
    return worst


def solve_refined(A, B, steps: int = 3):
    """Reference solution: GEPP solve plus a few steps of refinement with the double-double residual."""
    LU, ipiv, info = getrf(A)
    if info:
        raise ValueError("singular matrix (info=%d)" % info)
    X = getrs(LU, ipiv, B)
    for _ in range(steps):
        R = residual_dd(A, X, B)
        X = X + getrs(LU, ipiv, R)
    return X


def adjoint(A, x, xbar):
    """Reverse-mode adjoint of x = A^{-1} b: bbar = A^{-T} xbar, Abar = -bbar x^T."""
    LU, ipiv, info = getrf(A)
    if info:
        raise ValueError("singular matrix (info=%d)" % info)
    bbar = getrs(LU, ipiv, xbar, trans=True)
    for _ in range(2):
        bbar = bbar + getrs(LU, ipiv, residual_dd(A, bbar, xbar, trans=True), trans=True)
    Abar = -np.outer(bbar, x) if np.ndim(x) == 1 else -(_as2d(bbar) @ _as2d(x).T)
    return Abar, bbar


def householder_inverse(vs_left, vs_right, sigma):
    """Dense A^{-1} = H2^T diag(1/sigma) H1^T for A = H1 diag(sigma) H2 (see householder_solve), built by
    applying the reflectors to diag(1/sigma): O(n^2) per reflector.  Used for the exact kappa_inf."""
    n = len(sigma)
    M = np.diag(1.0 / np.asarray(sigma, dtype=np.float64))
    # rows: M <- M H1^T, the left reflectors last-to-first from the right (H1^T = Hd Hc Hb Ha)
    for v in reversed(vs_left):
        w = M @ v
        M -= np.outer(w, (2.0 / (v @ v)) * v)
    # columns: M <- H2^T M = Hd Hc Hb Ha M, so Ha acts first
    for v in vs_right:
        w = v @ M
        M -= np.outer((2.0 / (v @ v)) * v, w)
    return M


def householder_solve(vs_left, vs_right, sigma, b):
    """x = A^{-1} b for A = H1 diag(sigma) H2 with H1 = prod(H(v) for v in vs_left) in order and H2
    likewise, H(v) = I - 2 v v^T / (v^T v).  A^{-1} = H2^T diag(1/sigma) H1^T; reflectors are symmetric,
    so H1^T applies the left reflectors first-to-last and H2^T applies the right ones first-to-last."""
    x = np.array(b, dtype=np.float64, copy=True)
    for v in vs_left:
        x = x - (2.0 * (v @ x) / (v @ v)) * v
    x = x / sigma
    for v in vs_right:
        x = x - (2.0 * (v @ x) / (v @ v)) * v
    return x
