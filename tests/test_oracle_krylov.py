"""Pins of the Krylov oracle (oracle/krylov.py) against what the mathematics
fixes, independently of the oracle's own code:

* exact termination: in rational arithmetic CG (SPD), BiCG and BiCGSTAB reach
  the exact solution of an n x n system within n iterations (Sec. 2 states it
  for CG); the reference solution is an exact Gauss-Jordan solve written here;
* minimisation: the k-th CG iterate minimises the A-norm of the error over
  x0 + K_k(A, r0), the k-th GMRES iterate minimises the residual 2-norm over
  the same space (of the preconditioned system with left preconditioning), and
  a restarted cycle does so from the restart point; the references are
  least-squares solves over an explicit Krylov basis (numpy.linalg.lstsq);
* GMRES-based refinement on A = H1 diag(sigma) H2 reaches the closed-form
  solution within the backward-error bound.
A planted mistake in any of the recurrences (a sign, an index, a missing term)
breaks exact termination or the minimisation property."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import krylov


def frac_matrix(rows):
    return np.array([[Fraction(v) for v in r] for r in rows], dtype=object)


def exact_solve(A, b):
    n = len(b)
    M = [[Fraction(A[i, j]) for j in range(n)] + [Fraction(b[i])] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return np.array([M[i][n] / M[i][i] for i in range(n)], dtype=object)


SPD5 = [[10, 2, -1, 0, 3], [2, 9, 1, -2, 0], [-1, 1, 8, 1, -1], [0, -2, 1, 7, 2], [3, 0, -1, 2, 11]]
GEN5 = [[4, 1, -2, 0, 1], [3, 6, 0, 1, -1], [0, -2, 5, 2, 0], [1, 0, 3, 7, -2], [-2, 1, 0, 1, 5]]
B5 = [1, -2, 3, 0, 4]


def test_cg_exact_termination():
    A = frac_matrix(SPD5)
    b = np.array([Fraction(v) for v in B5], dtype=object)
    x, it, hist = krylov.cg(A, b, np.array([Fraction(0)] * 5, dtype=object), 0.0, 5)
    xs = exact_solve(A, b)
    assert it <= 5 and all(x[i] == xs[i] for i in range(5))
    assert hist[-1] == 0.0


def test_bicg_exact_termination():
    A = frac_matrix(GEN5)
    b = np.array([Fraction(v) for v in B5], dtype=object)
    x, it, hist = krylov.bicg(A, b, np.array([Fraction(0)] * 5, dtype=object), 0.0, 5)
    xs = exact_solve(A, b)
    assert it <= 5 and all(x[i] == xs[i] for i in range(5))


def test_bicgstab_exact_termination():
    A = frac_matrix(GEN5)
    b = np.array([Fraction(v) for v in B5], dtype=object)
    x, it, hist = krylov.bicgstab(A, b, np.array([Fraction(0)] * 5, dtype=object), 0.0, 5)
    xs = exact_solve(A, b)
    assert it <= 5 and all(x[i] == xs[i] for i in range(5))


def krylov_basis(A, r0, k):
    """An orthonormal basis of K_k(A, r0) = span{r0, A r0, ..., A^{k-1} r0}: each new direction is A
    times the newest basis vector, orthonormalised against the others by a library QR."""
    Q = (r0 / np.linalg.norm(r0))[:, None]
    for _ in range(k - 1):
        Q = np.linalg.qr(np.column_stack([Q, A @ Q[:, -1]]))[0]
    return Q


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_cg_minimises_the_energy_error(k):
    A = synth.spd_matrix(12, 3)
    b = synth.rng(4).uniform(-1, 1, 12)
    x, it, _ = krylov.cg(A, b, np.zeros(12), 0.0, k)
    assert it == k
    K = krylov_basis(A, b, k)
    y = np.linalg.solve(K.T @ A @ K, K.T @ b)
    assert np.max(np.abs(x - K @ y)) <= 1e-12 * np.max(np.abs(x))


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_gmres_minimises_the_residual(k):
    g = synth.rng(5)
    n = 10
    A = np.eye(n) + g.uniform(-1, 1, (n, n)) / 3
    b = g.uniform(-1, 1, n)
    x, it, hist = krylov.gmres(A, b, np.zeros(n), 20, 0.0, k)
    assert it == k
    K = krylov_basis(A, b, k)
    y = np.linalg.lstsq(A @ K, b, rcond=None)[0]
    xs = K @ y
    assert np.max(np.abs(x - xs)) <= 1e-11 * np.max(np.abs(xs))
    assert abs(hist[-1] - np.linalg.norm(b - A @ xs) / np.linalg.norm(b)) <= 1e-12


def test_gmres_restart_cycles():
    """GMRES(3) for 6 steps: two cycles, each the residual minimiser from its start."""
    g = synth.rng(6)
    n = 10
    A = np.eye(n) + g.uniform(-1, 1, (n, n)) / 3
    b = g.uniform(-1, 1, n)
    x, it, _ = krylov.gmres(A, b, np.zeros(n), 3, 0.0, 6)
    assert it == 6
    x1 = np.zeros(n)
    for _ in range(2):
        r = b - A @ x1
        K = krylov_basis(A, r, 3)
        x1 = x1 + K @ np.linalg.lstsq(A @ K, r, rcond=None)[0]
    assert np.max(np.abs(x - x1)) <= 1e-11 * np.max(np.abs(x1))


def test_gmres_left_preconditioned():
    g = synth.rng(7)
    n = 10
    A = np.eye(n) + g.uniform(-1, 1, (n, n)) / 2
    M = A + g.uniform(-1, 1, (n, n)) / 20
    Minv = np.linalg.inv(M)
    b = g.uniform(-1, 1, n)
    k = 4
    x, it, _ = krylov.gmres(A, b, np.zeros(n), 20, 0.0, k, prec=lambda v: Minv @ v)
    B = Minv @ A
    K = krylov_basis(B, Minv @ b, k)
    xs = K @ np.linalg.lstsq(B @ K, Minv @ b, rcond=None)[0]
    assert np.max(np.abs(x - xs)) <= 1e-10 * np.max(np.abs(xs))


def test_float_solvers_reach_tolerance():
    n = 200
    A = synth.spd_matrix(n, 8)
    b = synth.rng(9).uniform(-1, 1, n)
    x, it, hist = krylov.cg(A, b, np.zeros(n), 1e-12, 500)
    assert hist[-1] <= 1e-12 and np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-11
    G = np.eye(n) + synth.rng(10).uniform(-1, 1, (n, n)) / (2 * np.sqrt(n))
    for f in (krylov.bicg, krylov.bicgstab):
        x, it, hist = f(G, b, np.zeros(n), 1e-12, 500)
        assert np.linalg.norm(b - G @ x) / np.linalg.norm(b) <= 1e-11, f.__name__
    x, it, hist = krylov.gmres(G, b, np.zeros(n), 20, 1e-12, 500)
    assert np.linalg.norm(b - G @ x) / np.linalg.norm(b) <= 1e-11


@pytest.mark.parametrize("kappa", [1e4, 1e6])
def test_gmres_ir_reaches_the_closed_form_solution(kappa):
    """Preconditioner: FP32 GEPP factors with L and U rounded to BF16 (8 significant bits), far too
    coarse for classical refinement at this kappa; GMRES-IR still reaches eta <= 1e-14."""
    import torch
    n = 256
    A, xt, b, meta = synth.householder_system(n, kappa, seed=77)
    LU, ipiv, info = oracle.sgetrf(A)
    LUb = torch.from_numpy(np.asarray(LU, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    L, U = oracle.unpack_lu(LUb)
    perm = oracle.ipiv_to_perm(ipiv)

    def lu_solve(v):
        y = np.linalg.solve(L, v[perm])
        return np.linalg.solve(U, y)
    x, outer, inner, eta = krylov.gmres_ir(A, b, lu_solve)
    xs = oracle.householder_solve(meta["vs_left"], meta["vs_right"], meta["sigma"], b)
    assert eta <= 1e-14 and oracle.eta_inf(A, x, b) <= 1e-14
    assert np.max(np.abs(x - xs)) / np.max(np.abs(x)) <= n * kappa * 1e-14 + 64 * np.sqrt(n) * 2.0 ** -53


def test_bicgstab_first_step_minimises_over_omega():
    """One BiCGSTAB iteration from x0 = 0 is a BiCG step (alpha from the shadow-residual condition) and
    then the omega that minimises ||s - omega A s||_2 (library least squares)."""
    g = synth.rng(12)
    n = 9
    A = np.eye(n) + g.uniform(-1, 1, (n, n)) / 3
    b = g.uniform(-1, 1, n)
    x, it, _ = krylov.bicgstab(A, b, np.zeros(n), 0.0, 1)
    v = A @ b
    alpha = (b @ b) / (b @ v)
    s = b - alpha * v
    t = A @ s
    omega = np.linalg.lstsq(t[:, None], s, rcond=None)[0][0]
    xs = alpha * b + omega * s
    assert it == 1 and np.max(np.abs(x - xs)) <= 1e-13 * np.max(np.abs(xs))


def test_gmres_keeps_the_basis_orthogonal():
    """A spectrum over ten decades, n full GMRES steps: with the basis kept orthogonal the true
    residual falls below 1e-6 (one Gram-Schmidt pass loses orthogonality here and ends near 1)."""
    g = synth.rng(11)
    n = 60
    Q1 = np.linalg.qr(g.standard_normal((n, n)))[0]
    Q2 = np.linalg.qr(g.standard_normal((n, n)))[0]
    A = Q1 @ np.diag(np.logspace(0, -10, n)) @ Q2
    b = g.uniform(-1, 1, n)
    x, it, hist = krylov.gmres(A, b, np.zeros(n), 100, 0.0, n)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-6
