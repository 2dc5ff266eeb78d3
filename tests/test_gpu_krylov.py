"""Krylov solvers (CG, BiCG, BiCGSTAB, restarted GMRES) and GMRES-based
refinement on the GPU through the C-ABI, against the Krylov oracle
(oracle/krylov.py) on the same seeded inputs:

* a fixed number of iterations (tol = 0): the k-th iterate equals the
  oracle's element by element within rounding (the recurrences are the same;
  the dot products and matrix products add in another order);
* to convergence: the same iteration count within two, the true residual
  within ten times the tolerance, and the solution within the bound the
  tolerance implies;
* edge cases: n = 1, a size one row past a product block, an exact initial
  guess (zero iterations), b = 0;
* GMRES-based refinement with BF16 / FP16 factors at kappa = 1e6 reaching
  eta <= 1e-14 (the oracle's double-double check) and the closed-form
  Householder solution."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import krylov as ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cds():
    import paper_1511_07174_amd as m
    oracle.build()
    m.lib()
    return m


def dev():
    return torch.device("cuda", 0)


def to_dev(a):
    return torch.from_numpy(np.asfortranarray(a)).to(dev())


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def spd(n, seed):
    return synth.spd_matrix(n, seed)


def general(n, seed):
    """Well-conditioned nonsymmetric: I + R / (2 sqrt(n)), R ~ U[-1, 1]."""
    return np.asfortranarray(np.eye(n) + synth.rng(seed).uniform(-1, 1, (n, n)) / (2 * np.sqrt(n)))


ORACLE = {"cg": ok.cg, "bicg": ok.bicg, "bicgstab": ok.bicgstab}


def run(cds, method, A, b, **kw):
    prm = cds.cds.krylov_params(**kw)
    x, r = cds.krylov_solve(to_dev(A), to_dev(b), method, params=prm)
    return host(x), r


def oracle_run(method, A, b, tol, max_iter, restart=30):
    x0 = np.zeros(len(b))
    if method == "gmres":
        return ok.gmres(A, b, x0, restart, tol, max_iter)
    return ORACLE[method](A, b, x0, tol, max_iter)


@pytest.mark.parametrize("method", ["cg", "bicg", "bicgstab", "gmres"])
@pytest.mark.parametrize("k", [1, 3, 6])
def test_fixed_iterations_match_the_oracle(cds, method, k):
    n = 1000
    A = spd(n, 40) if method == "cg" else general(n, 41)
    b = synth.rng(42).uniform(-1, 1, n)
    x, r = run(cds, method, A, b, tol=0.0, max_iter=k, restart=4)
    xo, ito, hist = oracle_run(method, A, b, 0.0, k, restart=4)
    assert r.iters == ito == k, (r.iters, ito)
    assert np.max(np.abs(x - xo)) <= 1e-11 * np.max(np.abs(xo)), np.max(np.abs(x - xo))
    assert abs(r.relres - hist[-1]) <= 1e-9 * hist[-1] + 1e-300


@pytest.mark.parametrize("method", ["cg", "bicg", "bicgstab", "gmres"])
@pytest.mark.parametrize("n", [777, 2049])
def test_convergence_matches_the_oracle(cds, method, n):
    A = spd(n, 43) if method == "cg" else general(n, 44)
    b = synth.rng(45).uniform(-1, 1, n)
    tol = 1e-10
    x, r = run(cds, method, A, b, tol=tol, max_iter=500, restart=20)
    xo, ito, hist = oracle_run(method, A, b, tol, 500, restart=20)
    assert r.converged and not r.breakdown, r
    assert abs(r.iters - ito) <= 2, (r.iters, ito)
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert true <= 10 * tol, true
    # both solutions within their residuals of the exact one: ||x - xo|| <= ||A^-1|| (r + ro)
    assert np.max(np.abs(x - xo)) <= 1e-8 * np.max(np.abs(xo))


def test_edge_cases(cds):
    # n = 1
    x, r = run(cds, "cg", np.array([[4.0]]), np.array([2.0]), tol=1e-14, max_iter=10)
    assert r.converged and abs(x[0] - 0.5) <= 1e-15
    # exact initial guess: zero iterations
    n = 513
    A = spd(n, 46)
    xs = synth.rng(47).uniform(-1, 1, n)
    b = A @ xs
    for method in ("cg", "bicgstab", "gmres"):
        prm = cds.cds.krylov_params(tol=1e-6, max_iter=50)
        x0 = to_dev(xs)
        xg, rr = cds.krylov_solve(to_dev(A), to_dev(b), method, x0=x0, params=prm)
        assert rr.iters == 0 and rr.converged, (method, rr)
    # b = 0 gives x = 0
    for method in ("cg", "bicg", "bicgstab", "gmres"):
        x, r = run(cds, method, A, np.zeros(n), tol=1e-10, max_iter=20)
        assert r.converged and np.all(x == 0.0), (method, r)
    assert cds.handle().device_error() == 0


def test_check_every_zero_enqueues_the_budget(cds):
    """check_every = 0: no host reads; the iterations after convergence do nothing."""
    n = 600
    A = spd(n, 48)
    b = synth.rng(49).uniform(-1, 1, n)
    x1, r1 = run(cds, "cg", A, b, tol=1e-10, max_iter=200, check_every=0)
    x2, r2 = run(cds, "cg", A, b, tol=1e-10, max_iter=200, check_every=7)
    assert r1.converged and r1.iters == r2.iters
    assert np.array_equal(x1, x2)


@pytest.mark.parametrize("method", ["cg", "gmres"])
def test_full_size_16384(cds, method):
    n = 16384
    if method == "cg":
        A = synth.spd_matrix(n, synth.SEED_CHOL[n])
    else:
        A = general(n, 50)
    b = synth.rng(51).uniform(-1, 1, n)
    x, r = run(cds, method, A, b, tol=1e-10, max_iter=300, restart=30)
    xo, ito, hist = oracle_run(method, A, b, 1e-10, 300, restart=30)
    print("n=16384 %s: gpu %d iterations, oracle %d, relres %.2e" % (method, r.iters, ito, r.relres), flush=True)
    assert r.converged and abs(r.iters - ito) <= 2
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-9
    assert np.max(np.abs(x - xo)) <= 1e-8 * np.max(np.abs(xo))
    assert cds.handle().device_error() == 0


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_gmres_ir_householder(cds, prec):
    n = 2048
    kappa = 1e6
    A, xt, b, meta = synth.householder_system(n, kappa, seed=synth.householder_seed(8192, kappa))
    xs = oracle.householder_solve(meta["vs_left"], meta["vs_right"], meta["sigma"], b)
    x, r, inner = cds.solve_gmres_ir(to_dev(A), to_dev(b), precision=prec)
    x = host(x)
    eta = oracle.eta_inf(A, x, b)
    ferr = np.max(np.abs(x - xs)) / np.max(np.abs(x))
    print("GMRES-IR %s kappa=1e6: %d corrections, %d GMRES iterations, eta %.2e (oracle %.2e), fwd %.2e"
          % (prec, r.iters, inner, r.eta, eta, ferr), flush=True)
    assert r.info == 0 and r.converged, r
    assert eta <= 1e-14
    assert ferr <= n * kappa * eta * 1.01 + 64 * np.sqrt(n) * 2.0 ** -53
    assert inner > 0
    assert cds.handle().device_error() == 0
