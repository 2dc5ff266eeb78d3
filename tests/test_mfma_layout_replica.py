"""Host replica of the lane layouts behind the chained 16 x 16 x 4 MFMA products of the Cholesky
diagonal kernel (chol.hip, rows below a sub-block: X = B L^{-T} by 16 x 16 blocks) and of the FP64
panel's U_right (lu.hip: X = L^{-1} P).  An MFMA multiplies a 16 x 4 A by a 4 x 16 B: lane l holds
A(l % 16, l / 16) and B(l / 16, l % 16); accumulator v of lane l is D(4 (l / 16) + v, l % 16) for
FP32 and D(l / 16 + 4 v, l % 16) for FP64.  The kernels choose the k index of each k-step so that
one product's accumulators are the next product's B operand as they stand; the replica runs the
same lane-level steps with these layouts and must reproduce the blocked solves.  No GPU needed."""
import numpy as np
import pytest


def mfma(a, b, acc, f64):
    """One 16x16x4 step: a, b are per-lane values (64), acc per-lane 4-vectors (64 x 4)."""
    A = np.zeros((16, 4))
    B = np.zeros((4, 16))
    for l in range(64):
        A[l % 16, l // 16] = a[l]
        B[l // 16, l % 16] = b[l]
    D = A @ B
    out = acc.copy()
    for l in range(64):
        for v in range(4):
            i = (l // 16 + 4 * v) if f64 else (4 * (l // 16) + v)
            out[l, v] += D[i, l % 16]
    return out


def lanes():
    return np.arange(64) % 16, np.arange(64) // 16


def kidx(s, kl, f64):
    return 4 * s + kl if f64 else 4 * kl + s


def lower(g, n):
    L = np.tril(g.uniform(-0.5, 0.5, (n, n)), -1) + np.diag(g.uniform(1.0, 2.0, n))
    return L


@pytest.mark.parametrize("f64", [True, False])
def test_cholesky_rows_below(f64):
    """X0 = B0 inv(L00)^T, B1 -= X0 L10^T, X1 = B1 inv(L11)^T, with the kernel's operand choices."""
    g = np.random.default_rng(1 + f64)
    L = lower(g, 32)
    Bm = g.uniform(-1, 1, (16, 32))         # 16 rows of the tile, 32 columns of the sub-block
    inv0, inv1 = np.linalg.inv(L[:16, :16]), np.linalg.inv(L[16:, 16:])
    li, kl = lanes()
    x0 = np.zeros((64, 4))
    x1 = np.zeros((64, 4))
    b1 = np.array([[Bm[li[l], 16 + kidx(v, kl[l], f64)] for v in range(4)] for l in range(64)])
    for s in range(4):
        k = kidx(s, kl, f64)
        x0 = mfma(inv0[li, k], Bm[li, k], x0, f64)
    for s in range(4):
        k = kidx(s, kl, f64)
        b1 = mfma(-L[16 + li, k], x0[:, s], b1, f64)
    for s in range(4):
        k = kidx(s, kl, f64)
        x1 = mfma(inv1[li, k], b1[:, s], x1, f64)
    X = np.zeros((16, 32))
    for l in range(64):
        for v in range(4):
            X[li[l], kidx(v, kl[l], f64)] = x0[l, v]
            X[li[l], 16 + kidx(v, kl[l], f64)] = x1[l, v]
    assert np.allclose(X, Bm @ np.linalg.inv(L).T, rtol=0, atol=1e-12)


@pytest.mark.parametrize("t_f64", [True, False])
def test_panel_u_right(t_f64):
    """FP64 products with the inverses and an update in the factor's precision T: X0 = inv(L00) P0,
    P1 -= L10 X0, X1 = inv(L11) P1, for one 16-column tile; accumulators of the T product follow T's
    layout, and the last product takes its k index from that layout."""
    g = np.random.default_rng(7 + t_f64)
    L = np.tril(g.uniform(-0.5, 0.5, (32, 32)), -1) + np.eye(32)   # unit lower
    P = g.uniform(-1, 1, (32, 16))
    inv0, inv1 = np.linalg.inv(L[:16, :16]), np.linalg.inv(L[16:, 16:])
    li, kl = lanes()
    k64 = lambda v: kl + 4 * v
    kout = lambda v: (kl + 4 * v) if t_f64 else (4 * kl + v)
    x0 = np.zeros((64, 4))
    x1 = np.zeros((64, 4))
    p1 = np.array([[P[16 + kout(v)[l], li[l]] for v in range(4)] for l in range(64)])
    for s in range(4):
        x0 = mfma(inv0[li, k64(s)], P[k64(s), li], x0, True)
    for s in range(4):
        p1 = mfma(-L[16 + li, k64(s)], x0[:, s], p1, t_f64)
    for s in range(4):
        x1 = mfma(inv1[li, kout(s)], p1[:, s], x1, True)
    X = np.zeros((32, 16))
    for l in range(64):
        for v in range(4):
            X[k64(v)[l], li[l]] = x0[l, v]
            X[16 + k64(v)[l], li[l]] = x1[l, v]
    assert np.allclose(X, np.linalg.solve(L, P), rtol=0, atol=1e-12)


def test_mismatched_k_index_is_caught():
    # the FP32 layout with the FP64 k order: the chained operand no longer lines up
    g = np.random.default_rng(3)
    L = lower(g, 32)
    Bm = g.uniform(-1, 1, (16, 32))
    inv0 = np.linalg.inv(L[:16, :16])
    li, kl = lanes()
    x0 = np.zeros((64, 4))
    for s in range(4):
        k = kidx(s, kl, True)
        x0 = mfma(inv0[li, k], Bm[li, k], x0, False)
    X0 = np.zeros((16, 16))
    for l in range(64):
        for v in range(4):
            X0[li[l], kidx(v, kl[l], True)] = x0[l, v]
    assert not np.allclose(X0, Bm[:, :16] @ inv0.T, atol=1e-9)
