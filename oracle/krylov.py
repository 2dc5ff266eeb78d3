"""Plain CPU FP64 oracle of the Krylov solvers of arXiv 1511.07174 (Sec. 2):
conjugate gradient for SPD systems, GMRES restarted after a fixed number of
steps, BiCG (residual and shadow-residual sequences with A and A^T) and its
stabilised variant BiCGSTAB.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.
It shares no code with the HIP library.

Every function works on numpy arrays of float64, or of Python Fractions (object
arrays) for the exact-arithmetic pins; only +, -, *, / and the product @ are
used on the data, and the stopping test converts to float.  Conventions shared
with the GPU solvers:

* relative residual  rel_k = ||r_k||_2 / ||b||_2, with r_k the recurrence
  residual of the method; the solve stops at rel_k <= tol or after max_iter
  iterations (one iteration = one product with A, for BiCGSTAB one half step
  pair = two products, for BiCG one product with A and one with A^T);
* x0 is given (zero in the tests);
* GMRES orthogonalises the new Arnoldi vector by classical Gram-Schmidt
  applied twice (equal to modified Gram-Schmidt in exact arithmetic; the paper
  names only "Gram-Schmidt"), and solves the small least-squares problem with
  Givens rotations;
* left preconditioning for GMRES: M^{-1} A x = M^{-1} b through a callable
  `prec(v) = M^{-1} v`; its residual norms are those of the preconditioned
  system.
"""
from __future__ import annotations

import math

import numpy as np


def _dot(x, y):
    return x @ y


def _norm2(x) -> float:
    return math.sqrt(float(_dot(x, x)))


def cg(A, b, x0, tol: float, max_iter: int):
    """Conjugate gradient (Hestenes-Stiefel form).  Returns (x, iters, history) with history[k] =
    ||r_k|| / ||b|| for k = 0..iters."""
    x = x0.copy()
    r = b - A @ x
    p = r.copy()
    rr = _dot(r, r)
    nb = _norm2(b)
    hist = [_norm2(r) / nb]
    it = 0
    while it < max_iter and hist[-1] > tol:
        q = A @ p
        alpha = rr / _dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = _dot(r, r)
        it += 1
        hist.append(math.sqrt(float(rr_new)) / nb)
        if rr_new == 0:
            break
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    return x, it, hist


def bicg(A, b, x0, tol: float, max_iter: int):
    """BiConjugate gradient: residuals r (with A) and shadow residuals rt (with A^T), shadow start
    rt_0 = r_0.  Returns (x, iters, history)."""
    x = x0.copy()
    r = b - A @ x
    rt = r.copy()
    p = r.copy()
    pt = rt.copy()
    rho = _dot(rt, r)
    nb = _norm2(b)
    hist = [_norm2(r) / nb]
    it = 0
    At = A.T
    while it < max_iter and hist[-1] > tol:
        q = A @ p
        qt = At @ pt
        alpha = rho / _dot(pt, q)
        x = x + alpha * p
        r = r - alpha * q
        rt = rt - alpha * qt
        it += 1
        hist.append(_norm2(r) / nb)
        rho_new = _dot(rt, r)
        if rho_new == 0:
            break
        beta = rho_new / rho
        p = r + beta * p
        pt = rt + beta * pt
        rho = rho_new
    return x, it, hist


def bicgstab(A, b, x0, tol: float, max_iter: int):
    """BiCGSTAB (van der Vorst), shadow residual rh = r_0.  One iteration applies A twice.
    The stopping test is taken after the half step (on s) and after the full step (on r).
    Returns (x, iters, history) with history[k] = ||r_k|| / ||b||."""
    x = x0.copy()
    r = b - A @ x
    rh = r.copy()
    nb = _norm2(b)
    hist = [_norm2(r) / nb]
    rho = alpha = omega = None
    p = v = None
    it = 0
    while it < max_iter and hist[-1] > tol:
        rho_new = _dot(rh, r)
        if it == 0:
            p = r.copy()
        else:
            beta = (rho_new / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
        v = A @ p
        alpha = rho_new / _dot(rh, v)
        s = r - alpha * v
        it += 1
        if _norm2(s) / nb <= tol:
            x = x + alpha * p
            hist.append(_norm2(s) / nb)
            r = s
            break
        t = A @ s
        omega = _dot(t, s) / _dot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        hist.append(_norm2(r) / nb)
        rho = rho_new
    return x, it, hist


def _givens(a: float, b: float):
    """(c, s) with [c s; -s c] [a; b] = [h; 0], h = sqrt(a^2 + b^2)."""
    if b == 0.0:
        return 1.0, 0.0
    h = math.hypot(a, b)
    return a / h, b / h


def gmres(A, b, x0, restart: int, tol: float, max_iter: int, prec=None):
    """Restarted GMRES(restart) with classical Gram-Schmidt twice and Givens rotations.
    prec: callable v -> M^{-1} v (left preconditioning) or None.  One iteration = one Arnoldi step
    (one product with A, one application of prec).  Returns (x, iters, history): history[k] is the
    least-squares residual norm / ||M^{-1} b|| after k iterations (restarts recompute the true
    preconditioned residual)."""
    P = (lambda v: v) if prec is None else prec
    n = b.shape[0]
    x = np.array(x0, dtype=np.float64, copy=True)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(P(b)))
    r = P(b - A @ x)
    beta = float(np.linalg.norm(r))
    hist = [beta / nb]
    it = 0
    while it < max_iter and hist[-1] > tol:
        m = min(restart, max_iter - it)
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k_done = 0
        for k in range(m):
            w = P(A @ V[:, k])
            # classical Gram-Schmidt, twice
            h1 = V[:, :k + 1].T @ w
            w = w - V[:, :k + 1] @ h1
            h2 = V[:, :k + 1].T @ w
            w = w - V[:, :k + 1] @ h2
            hk = h1 + h2
            hn = float(np.linalg.norm(w))
            H[:k + 1, k] = hk
            H[k + 1, k] = hn
            # earlier rotations on the new column, then the new rotation
            for i in range(k):
                a_, b_ = H[i, k], H[i + 1, k]
                H[i, k] = cs[i] * a_ + sn[i] * b_
                H[i + 1, k] = -sn[i] * a_ + cs[i] * b_
            cs[k], sn[k] = _givens(H[k, k], H[k + 1, k])
            H[k, k] = cs[k] * H[k, k] + sn[k] * H[k + 1, k]
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            it += 1
            k_done = k + 1
            hist.append(abs(g[k + 1]) / nb)
            if hist[-1] <= tol or hn == 0.0:
                break
            V[:, k + 1] = w / hn
        # y = H^{-1} g by back substitution, x += V y
        kk = k_done
        y = np.zeros(kk)
        for i in range(kk - 1, -1, -1):
            s = g[i]
            for j in range(i + 1, kk):
                s -= H[i, j] * y[j]
            y[i] = s / H[i, i]
        x = x + V[:, :kk] @ y
        if hist[-1] <= tol or it >= max_iter:
            break
        r = P(b - A @ x)
        beta = float(np.linalg.norm(r))
        hist[-1] = beta / nb
    return x, it, hist


def gmres_ir(A, b, lu_solve, tol: float = 1e-14, inner_tol: float = 1e-4, restart: int = 30,
             max_outer: int = 20, max_inner: int = 60):
    """GMRES-based iterative refinement: x0 = lu_solve(b); then r = b - A x (FP64), solve A d = r
    by GMRES left-preconditioned with the low-precision factors (prec = lu_solve) to a relative
    preconditioned residual inner_tol, x += d, until the normwise backward error
    ||r||_inf / (||A||_inf ||x||_inf) <= tol.  Returns (x, outer, inner_total, eta)."""
    A = np.asarray(A, dtype=np.float64)
    nA = float(np.max(np.sum(np.abs(A), axis=1)))
    x = lu_solve(np.asarray(b, dtype=np.float64))
    inner_total = 0
    eta = math.inf
    for outer in range(max_outer + 1):
        r = b - A @ x
        eta = float(np.max(np.abs(r)) / (nA * np.max(np.abs(x))))
        if eta <= tol or outer == max_outer:
            return x, outer, inner_total, eta
        d, its, _ = gmres(A, r, np.zeros_like(r), restart, inner_tol, max_inner, prec=lu_solve)
        inner_total += its
        x = x + d
    return x, max_outer, inner_total, eta
