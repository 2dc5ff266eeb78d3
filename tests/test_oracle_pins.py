"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test fixes the oracle to something the paper's definitions (Sec. 2: A = LU
with unit lower L and partial pivoting, A = L L^T for SPD A, then Ly = b and
Ux = y) and elementary mathematics determine: exact constructions, closed forms,
exact rational arithmetic, invariants and finite differences.  A dropped term,
a wrong sign or index, or a transposed operand in the oracle fails at least one
of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import exact


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


# ---------------------------------------------------------------- exact constructions
@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (64, 3), (300, 4)])
def test_dyadic_plu_is_reproduced_bitwise(n, seed):
    A, L, U, perm = synth.dyadic_plu(n, seed)
    LU, ipiv, info = oracle.getrf(A)
    Lr, Ur = oracle.unpack_lu(LU)
    assert info == 0
    assert np.array_equal(Lr, L)
    assert np.array_equal(Ur, U)
    assert np.array_equal(ipiv, synth.perm_to_ipiv(perm))
    assert np.array_equal(oracle.ipiv_to_perm(ipiv), perm)
    # small-integer solution recovered exactly
    g = synth.rng(seed + 99)
    x = g.integers(-3, 4, size=n).astype(np.float64)
    b = A @ x
    assert np.array_equal(oracle.getrs(LU, ipiv, b), x)
    # transposed solve: A^T z = c with c = A^T x
    c = A.T @ x
    assert np.array_equal(oracle.getrs(LU, ipiv, c, trans=True), x)


@pytest.mark.parametrize("n", [2, 5, 30, 53])
def test_wilkinson_ties_take_lowest_index(n):
    A = synth.wilkinson(n)
    LU, ipiv, info = oracle.getrf(A)
    assert info == 0
    assert np.array_equal(ipiv, np.arange(1, n + 1))
    L, U = oracle.unpack_lu(LU)
    assert np.array_equal(U[:, n - 1], 2.0 ** np.arange(n))
    assert np.array_equal(np.tril(L, -1), -np.tril(np.ones((n, n)), -1))
    U_off = U[:, :n - 1]
    assert np.array_equal(U_off, np.eye(n)[:, :n - 1])


@pytest.mark.parametrize("n", [1, 2, 10, 29])
def test_pascal_cholesky_exact(n):
    A = synth.pascal(n)
    L, info = oracle.potrf(A)
    assert info == 0
    assert np.array_equal(np.tril(L), synth.pascal_factor(n))
    # strict upper triangle untouched
    assert np.array_equal(np.triu(L, 1), np.triu(A, 1))


def test_pascal_solve_small_integers():
    n = 12
    A = synth.pascal(n)
    L, _ = oracle.potrf(A)
    x = np.arange(-6, 6, dtype=np.float64)
    assert np.array_equal(oracle.potrs(L, A @ x), x)


@pytest.mark.parametrize("n", [1, 8, 100, 400])
def test_tridiag_closed_forms(n):
    T = synth.tridiag(n)
    L, info = oracle.potrf(T)
    assert info == 0
    d = np.diag(L)
    assert np.max(np.abs(d - synth.tridiag_cholesky_diag(n)) / d) < 8 * 2.0 ** -52
    # sub-diagonal l_{i+1,i} = -1 / l_ii (from l_{i+1,i} l_ii = -1)
    if n > 1:
        sub = np.diag(L, -1)
        assert np.max(np.abs(sub + 1.0 / d[:-1]) / np.abs(sub)) < 8 * 2.0 ** -52
    g = synth.rng(5)
    b = g.uniform(-1, 1, n)
    x_true = synth.tridiag_inverse(n) @ b
    x = oracle.potrs(L, b)
    kappa = np.linalg.norm(T, np.inf) * np.linalg.norm(synth.tridiag_inverse(n), np.inf)
    assert np.max(np.abs(x - x_true)) / np.max(np.abs(x_true)) < 4 * kappa * 2.0 ** -52 * n
    # LU path on the same matrix: no interchanges (diagonal dominance)
    LU, ipiv, info = oracle.getrf(T)
    assert info == 0 and np.array_equal(ipiv, np.arange(1, n + 1))


def test_trivial_matrices():
    n = 9
    LU, ipiv, info = oracle.getrf(np.eye(n))
    assert info == 0 and np.array_equal(LU, np.eye(n)) and np.array_equal(ipiv, np.arange(1, n + 1))
    D = np.diag(np.arange(1.0, n + 1))
    LU, ipiv, info = oracle.getrf(D)
    assert np.array_equal(LU, D) and np.array_equal(ipiv, np.arange(1, n + 1))
    perm = synth.rng(3).permutation(n)
    P = np.eye(n)[perm]          # P[k] = e_{perm[k]}: row k of P holds a 1 in column perm[k]
    LU, ipiv, info = oracle.getrf(P)
    Lr, Ur = oracle.unpack_lu(LU)
    assert info == 0 and np.array_equal(Lr, np.eye(n)) and np.array_equal(Ur, np.eye(n))
    assert np.array_equal(P[oracle.ipiv_to_perm(ipiv)], np.eye(n))
    # L = I - subdiagonal ones has L^{-1} = lower all-ones
    L = np.eye(n) - np.eye(n, k=-1)
    LU, ipiv, info = oracle.getrf(L)
    assert np.array_equal(ipiv, np.arange(1, n + 1))
    X = oracle.getrs(LU, ipiv, np.eye(n))
    assert np.array_equal(X, np.tril(np.ones((n, n))))
    # upper triangular: factors are A itself
    Ut = np.triu(synth.rng(4).integers(-4, 5, size=(n, n)).astype(float), 1) + 8 * np.eye(n)
    LU, ipiv, info = oracle.getrf(Ut)
    assert np.array_equal(LU, Ut) and np.array_equal(ipiv, np.arange(1, n + 1))


# ---------------------------------------------------------------- singular / non-SPD
def test_singular_cases():
    A = np.zeros((5, 5))
    LU, ipiv, info = oracle.getrf(A)
    assert info == 1 and np.array_equal(ipiv, np.arange(1, 6)) and not np.any(LU)
    g = synth.rng(7)
    A = g.uniform(-1, 1, (6, 6))
    A[4] = A[1]                   # equal rows -> rank 5, exact zero pivot at the last step
    A = np.round(A * 8) / 8       # dyadic entries keep the elimination exact enough to hit 0.0
    L, U, piv_x, info_x = exact.gepp(A)
    LU, ipiv, info = oracle.getrf(A)
    assert info_x > 0
    assert info == info_x
    A = np.diag([1.0, -1.0])
    L, info = oracle.potrf(A)
    assert info == 2
    A = np.diag([1.0, 0.0, 3.0])
    assert oracle.potrf(A)[1] == 2
    A = np.array([[4.0, 2.0], [2.0, 1.0]])   # PSD but singular: s = 1 - 1 = 0
    assert oracle.potrf(A)[1] == 2
    A = np.array([[np.nan, 0.0], [0.0, 1.0]])
    assert oracle.potrf(A)[1] == 1


def test_zero_column_continues():
    A = np.array([[0.0, 1.0, 2.0], [0.0, 2.0, 4.0], [0.0, 8.0, 3.0]])
    LU, ipiv, info = oracle.getrf(A)
    assert info == 1
    Lx, Ux, pivx, infox = exact.gepp(A)
    assert list(ipiv) == pivx
    assert np.array_equal(np.triu(LU), np.array([[float(v) for v in row] for row in Ux]))


# ---------------------------------------------------------------- brute force vs exact rationals
@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_exact_rationals(seed):
    g = synth.rng(100 + seed)
    n = int(g.integers(2, 8))
    A = g.integers(-9, 10, size=(n, n)).astype(np.float64)
    det = exact.det_leibniz(A)
    if det == 0:
        pytest.skip("singular draw")
    LU, ipiv, info = oracle.getrf(A)
    assert info == 0
    # pivots: compare with exact GEPP where the exact pivot choice is not a near tie
    Lx, Ux, pivx, infox = exact.gepp(A)
    if list(ipiv) != pivx:
        # allowed only when the exact pivot search had a tie in magnitude
        pytest.fail("pivot mismatch: oracle %s exact %s" % (list(ipiv), pivx))
    sign = 1
    for k in range(n):
        if ipiv[k] != k + 1:
            sign = -sign
    det_lu = sign * np.prod(np.diag(LU))
    assert abs(det_lu - float(det)) <= 1e-12 * abs(float(det)) + 1e-12
    b = g.integers(-9, 10, size=n).astype(np.float64)
    x = oracle.getrs(LU, ipiv, b)
    xs = exact.solve(A, b)
    r = exact.residual(A.tolist(), x.tolist(), b.tolist())
    eta = float(max(abs(v) for v in r)) / (np.max(np.sum(np.abs(A), 1)) * np.max(np.abs(x)))
    # kappa_inf from the exact inverse
    inv = [exact.solve(A, [1.0 if i == j else 0.0 for i in range(n)]) for j in range(n)]
    ninv = max(sum(abs(inv[j][i]) for j in range(n)) for i in range(n))
    kappa = float(ninv) * np.max(np.sum(np.abs(A), 1))
    fwd = max(abs(Fraction(x[i]) - xs[i]) for i in range(n)) / Fraction(np.max(np.abs(x)))
    assert float(fwd) <= kappa * eta * (1 + 1e-12) + 1e-300
    assert eta <= 1e-14
    # exact factors against the oracle's, to FP64 rounding
    Lf = np.array([[float(v) for v in row] for row in Lx])
    Uf = np.array([[float(v) for v in row] for row in Ux])
    L, U = oracle.unpack_lu(LU)
    assert np.max(np.abs(L - Lf)) <= 1e-13 * max(1.0, np.max(np.abs(Lf)))
    assert np.max(np.abs(U - Uf)) <= 1e-13 * max(1.0, np.max(np.abs(Uf)))


@pytest.mark.parametrize("seed", range(4))
def test_transposed_solve_vs_exact(seed):
    g = synth.rng(200 + seed)
    n = 6
    A = g.integers(-9, 10, size=(n, n)).astype(np.float64)
    if exact.det_leibniz(A) == 0:
        pytest.skip("singular draw")
    b = g.integers(-9, 10, size=n).astype(np.float64)
    LU, ipiv, _ = oracle.getrf(A)
    z = oracle.getrs(LU, ipiv, b, trans=True)
    zs = exact.solve(A.T.tolist(), b)
    assert max(abs(Fraction(z[i]) - zs[i]) for i in range(n)) <= Fraction(1, 10 ** 11) * max(1, max(abs(v) for v in zs))


@pytest.mark.parametrize("seed", range(4))
def test_cholesky_vs_exact_rational_solution(seed):
    g = synth.rng(300 + seed)
    n = 6
    M = g.integers(-5, 6, size=(n, n)).astype(np.float64)
    A = M @ M.T + n * np.eye(n)
    b = g.integers(-9, 10, size=n).astype(np.float64)
    L, info = oracle.potrf(A)
    assert info == 0
    x = oracle.potrs(L, b)
    xs = exact.solve(A.tolist(), b)
    assert max(abs(Fraction(x[i]) - xs[i]) for i in range(n)) <= Fraction(1, 10 ** 12) * max(1, max(abs(v) for v in xs))
    assert oracle.rho_llt(A, L) < 30


def test_residual_dd_is_correctly_rounded():
    g = synth.rng(11)
    for n in (3, 8):
        A = g.uniform(-1, 1, (n, n))
        x = g.uniform(-1, 1, n)
        b = A @ x + g.uniform(-1e-14, 1e-14, n)
        r = oracle.residual_dd(A, x, b)
        rx = exact.residual(A.tolist(), x.tolist(), b.tolist())
        for i in range(n):
            assert abs(Fraction(r[i]) - rx[i]) <= abs(rx[i]) * Fraction(2) ** -52
        rt = oracle.residual_dd(A, x, b, trans=True)
        rtx = exact.residual(A.T.tolist(), x.tolist(), b.tolist())
        for i in range(n):
            assert abs(Fraction(rt[i]) - rtx[i]) <= abs(rtx[i]) * Fraction(2) ** -52


# ---------------------------------------------------------------- random invariants (configs: n = 512)
def test_small_lu_workload_invariants():
    A, X, B = synth.uniform_system(512, 1, synth.SEED_SMALL_LU)
    LU, ipiv, info = oracle.getrf(A)
    assert info == 0
    x = oracle.getrs(LU, ipiv, B)
    assert oracle.eta_inf(A, x, B) <= 1e-14
    assert oracle.rho_lu(A, LU, ipiv) <= 30
    assert oracle.freivalds_lu(A, LU, ipiv) <= 1e-13
    # third-party library run (not read): same pivots, factors equal to rounding
    import scipy.linalg as sl
    lu, piv = sl.lu_factor(A)
    assert np.array_equal(piv + 1, ipiv)
    assert np.max(np.abs(lu - LU)) <= 1e-10


def test_planted_sign_error_is_caught():
    """A wrong sign in the rank-1 update breaks the dyadic pin (mutation check of the pins)."""
    A, L, U, perm = synth.dyadic_plu(16, 8)

    def bad_gepp(M):
        M = M.copy()
        n = M.shape[0]
        piv = []
        for k in range(n):
            mu = k + int(np.argmax(np.abs(M[k:, k])))
            piv.append(mu + 1)
            M[[k, mu]] = M[[mu, k]]
            M[k + 1:, k] /= M[k, k]
            M[k + 1:, k + 1:] += np.outer(M[k + 1:, k], M[k, k + 1:])   # planted: '+' for '-'
        return M, np.array(piv)

    LUb, pivb = bad_gepp(A)
    Lb, Ub = oracle.unpack_lu(LUb)
    assert not (np.array_equal(Lb, L) and np.array_equal(Ub, U))


# ---------------------------------------------------------------- generators and adjoint
def test_householder_construction_condition_and_inverse():
    n, kappa = 96, 1e4
    A, x_true, b, meta = synth.householder_system(n, kappa, seed=77)
    s = np.linalg.svd(A, compute_uv=False)
    assert abs(s[0] - 1.0) < 1e-12 and abs(s[-1] * kappa - 1.0) < 1e-8
    x = oracle.householder_solve(meta["vs_left"], meta["vs_right"], meta["sigma"], b)
    assert np.max(np.abs(x - x_true)) <= kappa * 1e-14
    xr = oracle.solve_refined(A, b)
    assert np.max(np.abs(xr - x)) <= kappa * 1e-14


def test_spd_generator_is_well_conditioned():
    A = synth.spd_matrix(300, 4)
    w = np.linalg.eigvalsh(A)
    assert w[0] >= 1.0 - 1e-12 and w[-1] <= 1.0 + 4.0 / 3.0 + 0.2
    L, info = oracle.potrf(A)
    assert info == 0 and oracle.rho_llt(A, L) < 30


def test_adjoint_matches_central_differences():
    """loss = w . x(A, b); dloss/db = A^{-T} w and dloss/dA = -bbar x^T, against central differences."""
    n = 64
    g = synth.rng(synth.SEED_FD)
    A = g.uniform(-1, 1, (n, n)) + 4 * np.eye(n)
    b = g.uniform(-1, 1, n)
    w = g.uniform(-1, 1, n)

    def loss(A_, b_):
        LU, ipiv, _ = oracle.getrf(A_)
        return float(w @ oracle.getrs(LU, ipiv, b_))

    x = oracle.solve_refined(A, b)
    Abar, bbar = oracle.adjoint(A, x, w)
    h = 1e-6
    for i in range(0, n, 7):
        e = np.zeros(n)
        e[i] = h
        fd = (loss(A, b + e) - loss(A, b - e)) / (2 * h)
        assert abs(fd - bbar[i]) <= 1e-7 * max(1.0, abs(bbar[i]))
    for (i, j) in [(0, 0), (3, 17), (63, 1), (20, 20), (40, 63)]:
        E = np.zeros((n, n))
        E[i, j] = h
        fd = (loss(A + E, b) - loss(A - E, b)) / (2 * h)
        assert abs(fd - Abar[i, j]) <= 1e-7 * max(1.0, abs(Abar[i, j]))


# ---------------------------------------------------------------- the checkers themselves
def _exact_eta(A, X, B):
    """Normwise backward error max_c ||b_c - A x_c||_inf / (||A||_inf ||x_c||_inf) in exact rationals."""
    n = A.shape[0]
    rows = [sum(abs(Fraction(float(A[i, j]))) for j in range(n)) for i in range(n)]
    nA = max(rows)
    worst = Fraction(0)
    for c in range(X.shape[1]):
        r = exact.residual(A.tolist(), X[:, c].tolist(), B[:, c].tolist())
        xm = max(abs(Fraction(float(v))) for v in X[:, c])
        worst = max(worst, max(abs(v) for v in r) / (nA * xm))
    return worst


@pytest.mark.parametrize("seed", range(6))
def test_eta_inf_equals_exact_rational(seed):
    """eta_inf (double-double residual, row-sum norm, max over |x| and over columns) against the same
    quantity in exact rational arithmetic: at most a few units of rounding apart."""
    g = synth.rng(400 + seed)
    n = int(g.integers(3, 8))
    A = g.integers(-9, 10, size=(n, n)).astype(np.float64)
    if exact.det_leibniz(A) == 0:
        A += 10 * np.eye(n)
    B = g.integers(-9, 10, size=(n, 3)).astype(np.float64)
    LU, ipiv, info = oracle.getrf(A)
    X = oracle.getrs(LU, ipiv, B)
    X[:, 1] *= 1.0 + 2.0 ** -40          # columns with different backward errors
    X[:, 2] += 2.0 ** -30
    ref = _exact_eta(A, X, B)
    got = oracle.eta_inf(A, X, B)
    assert ref > 0
    assert abs(Fraction(got) - ref) <= ref * Fraction(8) * Fraction(2) ** -52
    # transposed form: A^T x = b
    Xt = oracle.getrs(LU, ipiv, B, trans=True)
    Xt[:, 0] *= 1.0 - 2.0 ** -41
    ref_t = _exact_eta(A.T.copy(), Xt, B)
    got_t = oracle.eta_inf(A, Xt, B, trans=True)
    assert abs(Fraction(got_t) - ref_t) <= ref_t * Fraction(8) * Fraction(2) ** -52


def test_norm_inf_is_the_max_row_sum():
    """Hand matrices whose row sums, column sums and signed sums all differ."""
    A = np.array([[1.0, -10.0], [2.0, 0.0], [-3.0, 3.0]])      # rows 11, 2, 6; columns 6, 13
    assert oracle.norm_inf(A) == 11.0
    assert oracle.norm_inf(A.T) == 13.0
    B = np.array([[0.0, 5.0], [-4.0, -4.0]])                     # rows 5, 8; columns 4, 9; signed row sum -8
    assert oracle.norm_inf(B) == 8.0
    assert oracle.norm_inf(np.array([[-2.5]])) == 2.5
    assert np.isnan(oracle.norm_inf(np.array([[1.0, 0.0], [np.nan, 1.0]])))
    # eta picks the worst column, and divides by max |x| of that column, not of all of X
    A = np.eye(2)
    X = np.array([[1.0, 4.0], [0.5, 0.0]])
    B = np.array([[1.0, 4.0], [0.5, 1.0]])                       # column 1: r = (0, 1), ||x|| = 4
    assert oracle.eta_inf(A, X, B) == 0.25


def test_reconstruction_checkers_flag_planted_mistakes():
    """rho_lu, freivalds_lu and rho_llt are zero (to rounding) on exact factors and orders of magnitude
    above their thresholds when one entry of a factor is wrong, the permutation is dropped or
    inverted, or the factors are transposed."""
    n = 64
    A, L, U, perm = synth.dyadic_plu(n, 12)
    LU = np.tril(L, -1) + U
    ipiv = synth.perm_to_ipiv(perm)
    assert oracle.rho_lu(A, LU, ipiv) == 0.0
    assert oracle.freivalds_lu(A, LU, ipiv) <= 8 * oracle.EPS
    bad = LU.copy()
    bad[40, 7] += 2.0 ** -8                                      # one entry of L
    assert oracle.rho_lu(A, bad, ipiv) > 1e6
    assert oracle.freivalds_lu(A, bad, ipiv) > 1e-6
    bad = LU.copy()
    bad[3, 50] -= 2.0 ** -8                                      # one entry of U
    assert oracle.rho_lu(A, bad, ipiv) > 1e6
    assert oracle.freivalds_lu(A, bad, ipiv) > 1e-6
    ident = np.arange(1, n + 1, dtype=np.int32)                  # permutation dropped
    assert oracle.rho_lu(A, LU, ident) > 1e6
    assert oracle.freivalds_lu(A, LU, ident) > 1e-3
    inv = synth.perm_to_ipiv(np.argsort(perm))                   # permutation inverted
    assert oracle.rho_lu(A, LU, inv) > 1e6
    assert oracle.freivalds_lu(A, LU, inv) > 1e-3
    assert oracle.rho_lu(A, LU.T.copy(), ipiv) > 1e6            # transposed factors
    # Cholesky: the exact Pascal factor and a perturbed one
    P = synth.pascal(20)
    Lp = synth.pascal_factor(20)
    assert oracle.rho_llt(P, Lp) == 0.0
    badL = Lp.copy()
    badL[15, 3] += 1.0
    assert oracle.rho_llt(P, badL) > 1e6
    assert oracle.rho_llt(P, Lp.T.copy()) > 1e6                  # the upper triangle is ignored: L^T reads as diag only


@pytest.mark.parametrize("n,seed", [(1, 0), (9, 1), (64, 2), (300, 3)])
def test_sgetrf_dyadic_bitwise(n, seed):
    """The FP32 elimination reproduces the exact dyadic factors too: every intermediate of this
    construction is exact in single precision."""
    A, L, U, perm = synth.dyadic_plu(n, seed)
    LU, ipiv, info = oracle.sgetrf(A)
    assert LU.dtype == np.float32 and info == 0
    Lr, Ur = oracle.unpack_lu(LU.astype(np.float64))
    assert np.array_equal(Lr, L) and np.array_equal(Ur, U)
    assert np.array_equal(ipiv, synth.perm_to_ipiv(perm))


def test_sgetrf_is_single_precision_gepp():
    """Wilkinson ties (no interchange, U's last column 2^i), zero pivots as in FP64, and random FP32
    inputs: pivots of exact GEPP on the same FP32 values (no near ties), factors within FP32 rounding;
    the FP64 factors of the same input differ from them by far more than FP64 rounding."""
    W = synth.wilkinson(20)
    LU, ipiv, info = oracle.sgetrf(W)
    assert np.array_equal(ipiv, np.arange(1, 21)) and np.array_equal(LU[:, 19], 2.0 ** np.arange(20))
    Z = np.array([[0.0, 1.0, 2.0], [0.0, 2.0, 4.0], [0.0, 8.0, 3.0]])
    assert oracle.sgetrf(Z)[2] == oracle.getrf(Z)[2] == 1
    g = synth.rng(501)
    A = g.uniform(-1, 1, (7, 7)).astype(np.float32).astype(np.float64)
    Lx, Ux, pivx, _ = exact.gepp(A)
    LU, ipiv, info = oracle.sgetrf(A)
    assert list(ipiv) == pivx
    Uf = np.array([[float(v) for v in row] for row in Ux])
    Lf = np.array([[float(v) for v in row] for row in Lx])
    L32, U32 = oracle.unpack_lu(LU.astype(np.float64))
    scale = np.max(np.abs(Uf))
    assert np.max(np.abs(U32 - Uf)) <= 64 * 2.0 ** -24 * scale
    assert np.max(np.abs(L32 - Lf)) <= 64 * 2.0 ** -24 * max(1.0, np.max(np.abs(Lf)))
    LU64, _, _ = oracle.getrf(A)
    assert np.max(np.abs(LU64 - LU.astype(np.float64))) > 1e-12


def test_first_pivot_mismatch_reads_the_tie():
    """The pivot comparison helper: equal sequences report n; a sequence that takes the other row of
    an exact tie reports that step with multiplier 1; a wrong non-tied row reports |l| < 1."""
    A = np.array([[1.0, 2.0, 0.0], [-1.0, 0.0, 1.0], [0.5, 1.0, 3.0]])
    LU, ipiv, _ = oracle.getrf(A)
    assert oracle.first_pivot_mismatch(ipiv, LU, ipiv) == (3, 1.0)
    alt = ipiv.copy()
    alt[0] = 2                                                   # rows 0 and 1 tie at |1|
    k, mult = oracle.first_pivot_mismatch(alt, LU, ipiv)
    assert k == 0 and mult == 1.0
    alt = ipiv.copy()
    alt[0] = 3                                                   # row 2 has |0.5|: no tie
    k, mult = oracle.first_pivot_mismatch(alt, LU, ipiv)
    assert k == 0 and mult == 0.5


def test_freivalds_llt_flags_planted_mistakes():
    """Zero (to rounding) on the exact Pascal factor; far above the bar for a wrong entry, a transposed
    factor or a matrix whose upper triangle differs from its lower one (only the lower one is read)."""
    n = 24
    P = synth.pascal(n)
    Lp = synth.pascal_factor(n)
    assert oracle.freivalds_llt(P, Lp) <= 8 * oracle.EPS
    assert oracle.freivalds_llt(P, Lp.T.copy()) > 1e-3
    Pu = P.copy()
    Pu[0, n - 1] = 1e6                       # upper triangle ignored: still exact
    assert oracle.freivalds_llt(Pu, Lp) <= 8 * oracle.EPS
    S = synth.spd_matrix(200, 3)
    L, info = oracle.potrf(S)
    assert oracle.freivalds_llt(S, L) <= 1e-14
    bad = L.copy()
    bad[150, 30] += 1e-3                     # one wrong entry of L
    assert oracle.freivalds_llt(S, bad) > 1e-5
    bad = L.copy()
    bad[99, 99] *= 1.0 + 2.0 ** -20          # a diagonal entry off by a few parts per million
    assert oracle.freivalds_llt(S, bad) > 1e-8


def test_householder_inverse_and_condition():
    """The dense closed-form inverse inverts the stored matrix to rounding, its 2-norm condition is kappa,
    and the closed-form solution differs from the oracle's refined solve of the stored matrix by less
    than kappa_inf (eta + u): the bound the full-size forward-error checks use."""
    u = 2.0 ** -53
    for kappa in (1e2, 1e6):
        A, x_true, b, meta = synth.householder_system(512, kappa, seed=synth.householder_seed(8192, kappa))
        M = oracle.householder_inverse(meta["vs_left"], meta["vs_right"], meta["sigma"])
        assert np.max(np.abs(A @ M - np.eye(512))) <= kappa * 1e-13
        s = np.linalg.svd(M, compute_uv=False)
        assert abs(s[0] - kappa) <= 1e-8 * kappa and abs(s[-1] - 1.0) <= 1e-8
        kinf = oracle.norm_inf(A) * oracle.norm_inf(M)
        xs = oracle.householder_solve(meta["vs_left"], meta["vs_right"], meta["sigma"], b)
        xr = oracle.solve_refined(A, b)
        eta = oracle.eta_inf(A, xr, b)
        assert np.max(np.abs(xs - xr)) / np.max(np.abs(xr)) <= kinf * (eta + u)
        assert np.max(np.abs(M @ b - xs)) <= kinf * 4 * u * np.max(np.abs(xs))
