"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds none of the solver's arithmetic: it only draws random
numbers (numpy PCG64) and assembles test matrices whose factors or inverses
are known by construction.  Both the HIP path and the CPU oracle receive the
same FP64 bits from here.  Every array is returned in Fortran (column-major)
order.

Workloads (the paper's own test matrices are unspecified, so these stand in):

* ``uniform_system``   A ~ U[-1,1] i.i.d., X_true ~ U[-1,1], B = A X_true.
* ``spd_system``       A = M M^T / n + I with M ~ U[-1,1]  (SPD, kappa_2 <~ 2.4).
* ``householder_system``  A = H1 diag(sigma) H2, H1/H2 products of 4 Householder
  reflectors with N(0,1) vectors, sigma_i = kappa^(-i/(n-1)) (kappa_2(A) = kappa).
* ``vbatched_spd``     many SPD systems of sizes uniform in [nmin, nmax].
* exact constructions: ``dyadic_plu`` (A = P^T L U with dyadic L, U), ``wilkinson``,
  ``pascal``, ``tridiag``.
"""
from __future__ import annotations

import numpy as np

# seeds per workload family
SEED_SMALL_LU = 0
SEED_LU = {4096: 1, 8192: 2, 16384: 3}
SEED_CHOL = {4096: 4, 8192: 5, 16384: 6}
SEED_BATCH_GRAD = 20
SEED_FD = 21
SEED_VBATCH = 30


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def householder_seed(n: int, kappa: float) -> int:
    i_n = {8192: 0, 16384: 1, 32768: 2}.get(n, 0)
    i_k = {1e2: 0, 1e4: 1, 1e6: 2}.get(float(kappa), 0)
    return 10 + 3 * i_n + i_k


def _uniform_f(g, n, m):
    # draw column by column so that the values do not depend on memory order
    return np.asfortranarray(g.uniform(-1.0, 1.0, size=(m, n)).T)


def uniform_system(n: int, nrhs: int = 1, seed: int = 0):
    """(A, X_true, B) with A, X_true ~ U[-1,1] and B = A X_true."""
    g = rng(seed)
    A = _uniform_f(g, n, n)
    X = _uniform_f(g, n, nrhs)
    B = np.asfortranarray(A @ X)
    return A, X, B


def spd_matrix(n: int, seed: int):
    g = rng(seed)
    M = _uniform_f(g, n, n)
    A = (M @ M.T) / n
    A[np.diag_indices(n)] += 1.0
    return np.asfortranarray(A)


def spd_system(n: int, nrhs: int = 1, seed: int = 4):
    A = spd_matrix(n, seed)
    g = rng(seed + 1000)
    X = _uniform_f(g, n, nrhs)
    B = np.asfortranarray(A @ X)
    return A, X, B


def householder_system(n: int, kappa: float, seed: int | None = None, nrhs: int = 1):
    """A = H1 diag(sigma) H2 (kappa_2(A) = kappa exactly in exact arithmetic).

    Returns (A, x_true, b, meta) with meta = dict(vs_left, vs_right, sigma) so that the
    oracle can apply A^{-1} in O(n^2)."""
    if seed is None:
        seed = householder_seed(n, kappa)
    g = rng(seed)
    vs_left = [g.standard_normal(n) for _ in range(4)]
    vs_right = [g.standard_normal(n) for _ in range(4)]
    sigma = float(kappa) ** (-np.arange(n, dtype=np.float64) / max(1, n - 1))
    # H2 = Ha Hb Hc Hd, built by right-multiplying the identity by each reflector
    A = np.eye(n, dtype=np.float64, order="F")
    for v in vs_right:
        w = A @ v
        A -= np.outer(w, (2.0 / (v @ v)) * v)
    A *= sigma[:, None]
    # left factor: H1 A = Ha (Hb (Hc (Hd A)))
    for v in reversed(vs_left):
        w = v @ A
        A -= np.outer((2.0 / (v @ v)) * v, w)
    A = np.asfortranarray(A)
    X = _uniform_f(g, n, nrhs)
    B = np.asfortranarray(A @ X)
    if nrhs == 1:
        X, B = X[:, 0].copy(), B[:, 0].copy()
    return A, X, B, dict(vs_left=vs_left, vs_right=vs_right, sigma=sigma)


def vbatched_spd(count: int = 2000, nmin: int = 32, nmax: int = 1024, nrhs: int = 4, seed: int = SEED_VBATCH):
    """List of (A_i, B_i) SPD systems with n_i ~ U{nmin..nmax}; A_i = M M^T / n + I, B_i ~ U[-1,1]."""
    g = rng(seed)
    sizes = g.integers(nmin, nmax + 1, size=count)
    out = []
    for n in sizes:
        n = int(n)
        M = _uniform_f(g, n, n)
        A = (M @ M.T) / n
        A[np.diag_indices(n)] += 1.0
        B = _uniform_f(g, n, nrhs)
        out.append((np.asfortranarray(A), B))
    return out


def vbatched_sizes(count: int = 2000, nmin: int = 32, nmax: int = 1024, seed: int = SEED_VBATCH):
    g = rng(seed)
    return [int(v) for v in g.integers(nmin, nmax + 1, size=count)]


# ------------------------------------------------------------------------------
# exact constructions
# ------------------------------------------------------------------------------
def dyadic_plu(n: int, seed: int = 0):
    """A = P^T L U with unit-lower L (sub-diagonal in {0, +-1/4, +-1/2}), U with diagonal in
    {+-1, +-2, +-4} and off-diagonal integers in [-4, 4], and a random row permutation.

    Every quantity partial-pivoting elimination forms on this A is a small dyadic rational, so
    the factors are reproduced exactly under any summation order, with or without FMA.
    Returns (A, L, U, perm) where A = (L U)[inv(perm)], i.e. A[perm] = L U."""
    g = rng(seed)
    L = np.eye(n)
    sub = g.choice(np.array([0.0, 0.25, -0.25, 0.5, -0.5]), size=(n, n))
    L += np.tril(sub, -1)
    U = np.triu(g.integers(-4, 5, size=(n, n)).astype(np.float64), 1)
    U[np.diag_indices(n)] = g.choice(np.array([1.0, -1.0, 2.0, -2.0, 4.0, -4.0]), size=n)
    perm = g.permutation(n)
    LU = L @ U
    A = np.empty_like(LU)
    A[perm] = LU
    return np.asfortranarray(A), L, U, perm


def perm_to_ipiv(perm):
    """Sequential-interchange encoding (1-based) of the row order perm (A[perm] = P A)."""
    perm = np.asarray(perm)
    n = len(perm)
    cur = np.arange(n)           # cur[k] = original row now at position k
    where = np.arange(n)         # where[r] = current position of original row r
    ipiv = np.zeros(n, dtype=np.int32)
    for k in range(n):
        j = where[perm[k]]
        ipiv[k] = j + 1
        rk, rj = cur[k], cur[j]
        cur[k], cur[j] = rj, rk
        where[rk], where[rj] = j, k
    return ipiv


def wilkinson(n: int):
    """a_ii = 1, a_ij = -1 (i > j), last column all ones; partial pivoting takes no interchange
    (every candidate ties at |1|) and U's last column is 2^i (0-based i)."""
    A = np.eye(n) - np.tril(np.ones((n, n)), -1)
    A[:, n - 1] = 1.0
    return np.asfortranarray(A)


def pascal(n: int):
    """Symmetric Pascal matrix P_ij = C(i+j, i) = L L^T with L_ij = C(i, j) (0-based)."""
    from math import comb
    A = np.array([[comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)
    return np.asfortranarray(A)


def pascal_factor(n: int):
    from math import comb
    return np.array([[comb(i, j) if j <= i else 0 for j in range(n)] for i in range(n)], dtype=np.float64)


def tridiag(n: int):
    """tridiag(-1, 2, -1)."""
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return np.asfortranarray(A)


def tridiag_inverse(n: int):
    """(T^{-1})_ij = min(i, j) (n + 1 - max(i, j)) / (n + 1), 1-based indices."""
    i = np.arange(1, n + 1)
    mn = np.minimum.outer(i, i)
    mx = np.maximum.outer(i, i)
    return mn * (n + 1 - mx) / (n + 1)


def tridiag_cholesky_diag(n: int):
    """Diagonal of the Cholesky factor of tridiag(-1,2,-1): l_ii = sqrt((i+1)/i), 1-based i."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.sqrt((i + 1) / i)
