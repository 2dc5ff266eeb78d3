"""GPU parity of the HIP path against the CPU oracle, through the C-ABI.

Bars (written per test): bitwise for the exact constructions (dyadic P^T L U,
Wilkinson, Pascal, identity) and for pivot vectors where the oracle's pivot
choice has no near-tie; for random FP64 inputs the normwise backward error
eta_inf <= 1e-14, the reconstruction ratio rho <= 30, and the factors equal
to the oracle's within 1e-11 relative (blocked and unblocked elimination
differ only by rounding order: ~n eps growth).  FP32 factors use eps = 2^-23.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -23


@pytest.fixture(scope="module")
def cds():
    import paper_1511_07174_amd as m
    oracle.build()
    assert torch.cuda.is_available()
    m.lib()
    return m


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.asfortranarray(a)).to(dev(), dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def no_device_error(cds):
    assert cds.handle().device_error() == 0


# ------------------------------------------------------------------------ LU, exact constructions
@pytest.mark.parametrize("n", [1, 2, 31, 64, 300, 1000, 2100])
def test_getrf_dyadic_bitwise(cds, n):
    A, L, U, perm = synth.dyadic_plu(n, n)
    LU, ipiv, info = cds.getrf(to_dev(A))
    LUh = host(LU)
    Lr, Ur = oracle.unpack_lu(LUh)
    assert int(info.item()) == 0
    assert np.array_equal(host(ipiv), synth.perm_to_ipiv(perm))
    assert np.array_equal(Lr, L)
    assert np.array_equal(Ur, U)
    # exact integer solution, both op N and op T
    x = synth.rng(n + 5).integers(-3, 4, size=n).astype(np.float64)
    xs = cds.getrs(LU, ipiv, to_dev(A @ x))
    assert np.array_equal(host(xs), x)
    xt = cds.getrs(LU, ipiv, to_dev(A.T @ x), trans=True)
    assert np.array_equal(host(xt), x)
    no_device_error(cds)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nb,lookahead", [(32, 1), (64, 1), (128, 0), (192, 1), (384, 1), (512, 1), (512, 0)])
def test_getrf_block_sizes(cds, nb, lookahead, dtype):
    """Every block size (including the split TRSM beyond 384 FP64 rows) and both schedules give the
    exact factors of the dyadic construction."""
    from paper_1511_07174_amd.cds import OPT_NB, OPT_LOOKAHEAD
    n = 1100
    A, L, U, perm = synth.dyadic_plu(n, 77)
    h = cds.handle()
    h.set_option(OPT_NB, nb)
    h.set_option(OPT_LOOKAHEAD, lookahead)
    try:
        LU, ipiv, info = cds.getrf(to_dev(A, dtype))
        LUh = host(LU).astype(np.float64)
    finally:
        h.set_option(OPT_NB, 0)
        h.set_option(OPT_LOOKAHEAD, 1)
    Lr, Ur = oracle.unpack_lu(LUh)
    assert int(info.item()) == 0
    assert np.array_equal(host(ipiv), synth.perm_to_ipiv(perm))
    assert np.array_equal(Lr, L) and np.array_equal(Ur, U)
    no_device_error(cds)


@pytest.mark.parametrize("n", [5, 53])
def test_getrf_wilkinson_ties(cds, n):
    A = synth.wilkinson(n)
    LU, ipiv, info = cds.getrf(to_dev(A))
    LUo, ipo, _ = oracle.getrf(A)
    assert np.array_equal(host(ipiv), np.arange(1, n + 1))
    assert np.array_equal(host(LU), LUo)


def test_getrf_identity_and_zero(cds):
    n = 130
    LU, ipiv, info = cds.getrf(to_dev(np.eye(n)))
    assert np.array_equal(host(LU), np.eye(n)) and int(info.item()) == 0
    LU, ipiv, info = cds.getrf(to_dev(np.zeros((n, n))))
    assert int(info.item()) == 1
    assert np.array_equal(host(ipiv), np.arange(1, n + 1))
    assert not np.any(host(LU))


def test_getrf_singular_equal_rows(cds):
    g = synth.rng(7)
    A = np.round(g.uniform(-1, 1, (40, 40)) * 8) / 8
    A[33] = A[5]
    LUo, ipo, info_o = oracle.getrf(A)
    LU, ipiv, info = cds.getrf(to_dev(A))
    assert info_o > 0
    assert int(info.item()) == info_o


# ------------------------------------------------------------------------ LU, random (the small LU workload)
@pytest.mark.parametrize("n,seed", [(512, synth.SEED_SMALL_LU), (777, 3), (1500, 4)])
def test_getrf_random_vs_oracle(cds, n, seed):
    A, X, B = synth.uniform_system(n, 1, seed)
    LU, ipiv, info = cds.getrf(to_dev(A))
    LUo, ipo, info_o = oracle.getrf(A)
    LUh, ph = host(LU), host(ipiv)
    assert int(info.item()) == 0
    mism = int(np.sum(ph != ipo))
    assert mism == 0, "pivot mismatches: %d" % mism
    assert np.max(np.abs(LUh - LUo)) <= 1e-11 * np.max(np.abs(LUo))
    assert oracle.rho_lu(A, LUh, ph) <= 30
    x = cds.getrs(LU, ipiv, to_dev(B[:, 0]))
    assert oracle.eta_inf(A, host(x), B[:, 0]) <= 1e-14
    no_device_error(cds)


@pytest.mark.parametrize("nrhs", [1, 7, 32, 33])
@pytest.mark.parametrize("trans", [False, True])
def test_getrs_multi_rhs(cds, nrhs, trans):
    n = 700
    A, X, B = synth.uniform_system(n, nrhs, 11)
    LU, ipiv, info = cds.getrf(to_dev(A))
    Bt = (A.T @ X) if trans else B
    Xd = cds.getrs(LU, ipiv, to_dev(Bt), trans=trans)
    Xh = host(Xd)
    assert oracle.eta_inf(A, Xh, Bt, trans=trans) <= 1e-14
    Xo = oracle.getrs(host(LU), host(ipiv), Bt, trans=trans)
    assert np.max(np.abs(Xh - Xo)) <= 1e-10 * np.max(np.abs(Xo))


def test_sgetrf_fp32_invariants(cds):
    n = 900
    A, X, B = synth.uniform_system(n, 1, 12)
    A32 = A.astype(np.float32)
    LU, ipiv, info = cds.getrf(to_dev(A32, torch.float32))
    assert int(info.item()) == 0
    LUh = host(LU).astype(np.float64)
    assert oracle.rho_lu(A32.astype(np.float64), LUh, host(ipiv), eps=EPS32) <= 30
    b32 = B[:, 0].astype(np.float32)
    x = cds.getrs(LU, ipiv, to_dev(b32, torch.float32))
    eta = oracle.eta_inf(A32.astype(np.float64), host(x).astype(np.float64), b32.astype(np.float64))
    assert eta <= 30 * EPS32


def test_sgetrf_dyadic_bitwise(cds):
    n = 400
    A, L, U, perm = synth.dyadic_plu(n, 2)
    LU, ipiv, info = cds.getrf(to_dev(A, torch.float32))
    Lr, Ur = oracle.unpack_lu(host(LU).astype(np.float64))
    assert np.array_equal(host(ipiv), synth.perm_to_ipiv(perm))
    assert np.array_equal(Lr, L) and np.array_equal(Ur, U)


def test_getrf_strided_batched(cds):
    n, batch = 300, 5
    As = [synth.uniform_system(n, 1, 40 + b)[0] for b in range(batch)]
    Ad = torch.stack([to_dev(a) for a in As])
    LU, ipiv, info = cds.getrf(Ad)
    for b in range(batch):
        LUo, ipo, _ = oracle.getrf(As[b])
        assert np.array_equal(host(ipiv[b]), ipo)
        assert np.max(np.abs(host(LU[b]) - LUo)) <= 1e-11 * np.max(np.abs(LUo))
    assert not np.any(host(info))


# ------------------------------------------------------------------------ Cholesky
@pytest.mark.parametrize("n", [1, 10, 29])
def test_potrf_pascal_bitwise(cds, n):
    A = synth.pascal(n)
    L, info = cds.potrf(to_dev(A))
    Lh = host(L)
    assert int(info.item()) == 0
    assert np.array_equal(np.tril(Lh), synth.pascal_factor(n))
    assert np.array_equal(np.triu(Lh, 1), np.triu(A, 1))


@pytest.mark.parametrize("n", [200, 1000, 2100])
def test_potrf_spd_vs_oracle(cds, n):
    A = synth.spd_matrix(n, 4)
    L, info = cds.potrf(to_dev(A))
    Lh = host(L)
    Lo, info_o = oracle.potrf(A)
    assert int(info.item()) == 0 and info_o == 0
    assert np.max(np.abs(np.tril(Lh) - np.tril(Lo))) <= 1e-12 * np.max(np.abs(np.tril(Lo)))
    assert np.array_equal(np.triu(Lh, 1), np.triu(A, 1))
    assert oracle.rho_llt(A, Lh) <= 30
    g = synth.rng(9)
    B = g.uniform(-1, 1, (n, 3))
    X = cds.potrs(L, to_dev(B))
    assert oracle.eta_inf(A, host(X), B) <= 1e-14


def test_potrf_not_spd(cds):
    A = synth.spd_matrix(300, 5)
    A[150, 150] = -5.0
    Lo, info_o = oracle.potrf(A)
    L, info = cds.potrf(to_dev(A))
    assert info_o > 0 and int(info.item()) == info_o
    A = np.diag([1.0, -1.0])
    L, info = cds.potrf(to_dev(A))
    assert int(info.item()) == 2


def test_tridiag_potrs_closed_form(cds):
    n = 500
    T = synth.tridiag(n)
    L, info = cds.potrf(to_dev(T))
    d = np.diag(host(L))
    assert np.max(np.abs(d - synth.tridiag_cholesky_diag(n)) / d) <= 8 * 2.0 ** -52
    b = synth.rng(5).uniform(-1, 1, n)
    x = host(cds.potrs(L, to_dev(b)))
    x_true = synth.tridiag_inverse(n) @ b
    kappa = 4.0 * np.linalg.norm(synth.tridiag_inverse(n), np.inf)
    assert np.max(np.abs(x - x_true)) / np.max(np.abs(x_true)) <= kappa * 1e-15 * n


# ------------------------------------------------------------------------ mixed precision + refinement
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_gesv_mixed_householder_kappa100(cds, prec):
    n = 1024
    A, x_true, b, meta = synth.householder_system(n, 1e2, seed=77)
    X, res = cds.solve(to_dev(A), to_dev(b), precision=prec)
    r = res[0]
    x = host(X)
    assert r.converged and r.info == 0, r
    eta = oracle.eta_inf(A, x, b)
    assert eta <= 1e-14
    xs = oracle.householder_solve(meta["vs_left"], meta["vs_right"], meta["sigma"], b)
    fwd = np.max(np.abs(x - xs)) / np.max(np.abs(x))
    assert fwd <= 1e2 * 1e-13
    no_device_error(cds)


def test_gesv_mixed_uniform(cds):
    n = 2000
    A, X, B = synth.uniform_system(n, 1, 13)
    Xd, res = cds.solve(to_dev(A), to_dev(B[:, 0]), precision="fp32")
    assert res[0].converged, res[0]
    assert oracle.eta_inf(A, host(Xd), B[:, 0]) <= 1e-14


def test_block_inverse_first_solve(cds):
    """The refinement solves one right-hand side with the FP32 factors through 128 x 128 diagonal-block
    inverses.  With no refinement step (max_iter = 0) the result is that solve's x0, and its residual
    against the same factors, ||P b - L U x0|| / (|| |L| |U| || ||x0||) (infinity norms), is held to
    8 * 128 * u32 * max_b cond(D_b) over the diagonal blocks D_b of L and U: a block solved through an
    explicit inverse leaves a residual of at most about 2 * 128 * u * cond(D_b) ||v||, for each of the two
    triangles, with a factor 2 of margin.  n = 1000 spans seven full blocks and a ragged one."""
    n = 1000
    A, _, B = synth.uniform_system(n, 1, 31)
    b = B[:, 0]
    d = dev()
    Ad = cds.colmajor(to_dev(A))
    X = torch.zeros(n, dtype=torch.float64, device=d)
    LU = torch.empty(n * n, dtype=torch.float32, device=d)
    ipiv = torch.zeros(n, dtype=torch.int32, device=d)
    res = torch.zeros(cds.cds.IR_RESULT_BYTES, dtype=torch.uint8, device=d)
    cds.handle().gesv_mixed(Ad, to_dev(b), X, LU, ipiv, res, precision="fp32",
                            params=cds.default_params(max_iter=0))
    x0 = host(X)
    F = host(LU).astype(np.float64).reshape(n, n).T     # column-major storage
    L, U = oracle.unpack_lu(F)
    perm = oracle.ipiv_to_perm(host(ipiv))
    r = b[perm] - L @ (U @ x0)
    eta = np.max(np.abs(r)) / (np.max(np.sum(np.abs(L) @ np.abs(U), axis=1)) * np.max(np.abs(x0)))
    kmax = 0.0
    for k in range(0, n, 128):
        e = min(n, k + 128)
        for T in (L[k:e, k:e], U[k:e, k:e]):
            kmax = max(kmax, np.linalg.norm(T, np.inf) * np.linalg.norm(np.linalg.inv(T), np.inf))
    assert eta <= 8 * 128 * 2.0 ** -24 * kmax, (eta, kmax)
    no_device_error(cds)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_posv_mixed(cds, prec):
    n = 800
    A, X, B = synth.spd_system(n, 2, 6)
    Xd, res = cds.solve(to_dev(A), to_dev(B), precision=prec, spd=True)
    assert res[0].converged, res[0]
    assert oracle.eta_inf(A, host(Xd), B) <= 1e-14


@pytest.mark.parametrize("nb", [128, 160, 192])
def test_spotrf_block_sizes(cds, nb):
    """FP32 Cholesky with the diagonal block in LDS up to 192 columns (FP32 only): the factor of the
    FP32-rounded matrix has a backward error of a few FP32 units (the bound of the FP64 test, in
    FP32's epsilon), agrees with the oracle's factor to FP32 accuracy, and the mixed solves (FP32
    and FP16-operand factors) with the same block size converge to the FP64 bar."""
    from paper_1511_07174_amd.cds import OPT_NB
    n = 700
    A = synth.spd_matrix(n, 12)
    A32 = A.astype(np.float32).astype(np.float64)
    B = synth.rng(13).uniform(-1, 1, (n, 2))
    h = cds.handle()
    h.set_option(OPT_NB, nb)
    try:
        L, info = cds.potrf(to_dev(A32, torch.float32))
        sols = [cds.solve(to_dev(A), to_dev(B), precision=p, spd=True) for p in ("fp32", "fp16")]
    finally:
        h.set_option(OPT_NB, 0)
    Lh = np.tril(host(L).astype(np.float64))
    Lo, info_o = oracle.potrf(A32)
    assert int(info.item()) == 0 and info_o == 0
    assert oracle.rho_llt(A32, Lh, eps=EPS32) <= 30
    assert np.max(np.abs(Lh - np.tril(Lo))) <= 1e3 * EPS32 * np.max(np.abs(np.tril(Lo)))
    for Xd, res in sols:
        assert res[0].converged, res[0]
        assert oracle.eta_inf(A, host(Xd), B) <= 1e-14
    no_device_error(cds)


@pytest.mark.parametrize("spd", [False, True])
def test_fp16_operand_scale_is_exact(cds, spd):
    """The FP16 update multiplies op(B) by a power of two taken from max|op(B)| and the product by its
    inverse.  Every scaling on the path is then exact, so the system times 2^-24 must give the bitwise
    same solution and step count as the system itself (a scale taken from the wrong block, or not
    undone, breaks this; without the scale 2^-24 U12 would fall below FP16's normal range)."""
    n = 1200
    if spd:
        A, _, B = synth.spd_system(n, 1, 21)
        b = B[:, 0]
    else:
        A, _, b, _ = synth.householder_system(n, 1e2, seed=21)
    s = 2.0 ** -24
    x1, r1 = cds.solve(to_dev(A), to_dev(b), precision="fp16", spd=spd)
    x2, r2 = cds.solve(to_dev(A * s), to_dev(b * s), precision="fp16", spd=spd)
    assert r1[0].converged and r2[0].converged, (r1[0], r2[0])
    assert r1[0].iters == r2[0].iters
    assert np.array_equal(host(x1), host(x2))
    no_device_error(cds)


# ------------------------------------------------------------------------ differentiable solve
def test_solve_adjoint_matches_oracle(cds):
    n = 64
    g = synth.rng(synth.SEED_FD)
    A = g.uniform(-1, 1, (n, n)) + 4 * np.eye(n)
    b = g.uniform(-1, 1, n)
    w = g.uniform(-1, 1, n)
    Ad = to_dev(A).requires_grad_(True)
    bd = to_dev(b).requires_grad_(True)
    x = cds.solve_ad(Ad, bd)
    loss = (x * to_dev(w)).sum()
    loss.backward()
    xo = oracle.solve_refined(A, b)
    Abar_o, bbar_o = oracle.adjoint(A, xo, w)
    assert np.max(np.abs(host(bd.grad) - bbar_o)) <= 1e-12 * np.max(np.abs(bbar_o))
    assert np.max(np.abs(host(Ad.grad) - Abar_o)) <= 1e-12 * np.max(np.abs(Abar_o))


# ------------------------------------------------------------------------ batched uneven SPD
def test_vbatched_small(cds):
    sizes = [33, 1, 64, 100, 257, 31]
    g = synth.rng(3)
    systems = []
    host_sys = []
    for n in sizes:
        M = g.uniform(-1, 1, (n, n))
        A = M @ M.T / n + np.eye(n)
        B = g.uniform(-1, 1, (n, 4))
        host_sys.append((A, B))
        systems.append((to_dev(A), to_dev(B)))
    Xs, res, t0, t1 = cds.solve_vbatched(systems, nrhs=4)
    for (A, B), X, r in zip(host_sys, Xs, res):
        assert r.info == 0 and r.converged, r
        assert oracle.eta_inf(A, host(X), B) <= 1e-14
    no_device_error(cds)
