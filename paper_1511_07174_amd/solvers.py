"""Functional API over the C-ABI: factorizations, solves, mixed precision,
batched uneven SPD systems, and the differentiable solve.

The direct method of arXiv 1511.07174, Sec. 2: A = LU with partial pivoting
(A = L L^T for SPD A), then Ly = b and Ux = y.  All arithmetic runs in the
library's HIP kernels; these functions allocate outputs (torch tensors), make
column-major copies where needed and call the library.
"""
from __future__ import annotations

import torch

from . import cds
from .cds import colmajor, IrParams, default_params, decode_results


def _h():
    return cds.handle()


def getrf(A: torch.Tensor):
    """LU with partial pivoting of a square matrix (or a batch (b, n, n)).

    Returns (LU, ipiv, info): LU column-major, ipiv 1-based int32, info int32."""
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("getrf: float64 or float32 expected")
    LU = colmajor(A)
    n = A.shape[-1]
    if A.dim() == 3:
        ipiv = torch.zeros(A.shape[0], n, dtype=torch.int32, device=A.device)
        info = torch.zeros(A.shape[0], dtype=torch.int32, device=A.device)
    else:
        ipiv = torch.zeros(n, dtype=torch.int32, device=A.device)
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _h().getrf_(LU, ipiv, info)
    return LU, ipiv, info


def getrs(LU: torch.Tensor, ipiv: torch.Tensor, B: torch.Tensor, trans: bool = False):
    """Solve A X = B (or A^T X = B) from getrf's factors; returns a new column-major X."""
    X = colmajor(B) if B.dim() == LU.dim() else B.clone()
    _h().getrs_(LU, ipiv, X, trans=trans)
    return X


def potrf(A: torch.Tensor):
    """Lower Cholesky; returns (L, info).  The strict upper triangle is a copy of A's."""
    L = colmajor(A)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _h().potrf_(L, info)
    return L, info


def potrs(L: torch.Tensor, B: torch.Tensor):
    X = colmajor(B) if B.dim() == 2 else B.clone()
    _h().potrs_(L, X)
    return X


def solve(A: torch.Tensor, B: torch.Tensor, precision: str = "fp64", params: IrParams | None = None,
          spd: bool = False):
    """x = A^{-1} b.  precision "fp64": getrf + getrs (potrf + potrs when spd).
    "fp32" / "bf16" / "fp16": low-precision factorization with FP64 refinement.
    Returns (X, info_or_results)."""
    A = A.to(torch.float64) if precision != "fp64" else A
    if precision == "fp64":
        if spd:
            L, info = potrf(A)
            return potrs(L, B), info
        LU, ipiv, info = getrf(A)
        return getrs(LU, ipiv, B), info
    Ac = colmajor(A)
    Bc = colmajor(B) if B.dim() == A.dim() else B.contiguous()
    X = torch.zeros_like(Bc)
    X = colmajor(X) if X.dim() == A.dim() else X
    n = A.shape[-1]
    batch = A.shape[0] if A.dim() == 3 else 1
    res = torch.zeros(batch * cds.IR_RESULT_BYTES, dtype=torch.uint8, device=A.device)
    if spd:
        Llo = torch.empty(n * n, dtype=torch.float32, device=A.device)
        _h().posv_mixed(Ac, Bc, X, Llo, res, precision=precision, params=params)
        return X, decode_results(res)
    LUlo = torch.empty((batch, n * n) if batch > 1 or A.dim() == 3 else (n * n,), dtype=torch.float32,
                       device=A.device)
    ipiv = torch.zeros((batch, n) if A.dim() == 3 else (n,), dtype=torch.int32, device=A.device)
    _h().gesv_mixed(Ac, Bc, X, LUlo, ipiv, res, precision=precision, params=params)
    return X, decode_results(res)


def krylov_solve(A: torch.Tensor, b: torch.Tensor, method: str = "cg", x0: torch.Tensor | None = None,
                 params: cds.KrylovParams | None = None):
    """Krylov solve of A x = b in FP64 ("cg", "bicg", "bicgstab", "gmres"); returns (x, KrylovResult)."""
    Ac = colmajor(A.to(torch.float64))
    bc = b.to(torch.float64).contiguous()
    x = torch.zeros_like(bc) if x0 is None else x0.to(torch.float64).clone()
    res = torch.zeros(cds.KRYLOV_RESULT_BYTES, dtype=torch.uint8, device=A.device)
    _h().krylov(method, Ac, bc, x, res, params)
    return x, cds.decode_krylov(res)


def solve_gmres_ir(A: torch.Tensor, b: torch.Tensor, precision: str = "bf16", params: IrParams | None = None,
                   inner: cds.KrylovParams | None = None):
    """GMRES-based refinement: low-precision LU, FP64 GMRES corrections preconditioned by it.
    Returns (x, IrResult, total GMRES iterations)."""
    Ac = colmajor(A.to(torch.float64))
    bc = b.to(torch.float64).contiguous()
    n = A.shape[-1]
    x = torch.zeros_like(bc)
    LUlo = torch.empty(n * n, dtype=torch.float32, device=A.device)
    ipiv = torch.zeros(n, dtype=torch.int32, device=A.device)
    res = torch.zeros(cds.IR_RESULT_BYTES, dtype=torch.uint8, device=A.device)
    _h().gesv_gmres_ir(Ac, bc, x, LUlo, ipiv, res, precision=precision, params=params, inner=inner)
    inner_its = int(res.cpu()[36:40].view(torch.int32).item())
    return x, decode_results(res)[0], inner_its


def solve_vbatched(systems, nrhs: int = 4, params: IrParams | None = None, order=None, device="cuda"):
    """Many SPD systems of uneven size in one persistent launch (FP32 Cholesky, FP64 refinement).

    systems: list of (A_i, B_i) device float64 tensors (A_i column-major n_i x n_i, B_i n_i x nrhs).
    Returns (X list, results list, t_start, t_end)."""
    batch = len(systems)
    dev = torch.device(device)
    ns = torch.tensor([a.shape[0] for a, _ in systems], dtype=torch.int32, device=dev)
    Ap = torch.tensor([a.data_ptr() for a, _ in systems], dtype=torch.int64, device=dev)
    lda = torch.tensor([max(1, a.stride(1)) for a, _ in systems], dtype=torch.int64, device=dev)
    Bp = torch.tensor([b.data_ptr() for _, b in systems], dtype=torch.int64, device=dev)
    ldb = torch.tensor([max(1, b.stride(1)) if b.dim() == 2 else b.shape[0] for _, b in systems], dtype=torch.int64,
                       device=dev)
    Xs = [colmajor(torch.zeros_like(b)) for _, b in systems]
    Xp = torch.tensor([x.data_ptr() for x in Xs], dtype=torch.int64, device=dev)
    ldx = torch.tensor([max(1, x.stride(1)) if x.dim() == 2 else x.shape[0] for x in Xs], dtype=torch.int64,
                       device=dev)
    nmax = int(max(a.shape[0] for a, _ in systems))
    res = torch.zeros(batch * cds.IR_RESULT_BYTES, dtype=torch.uint8, device=dev)
    t0 = torch.zeros(batch, dtype=torch.int64, device=dev)
    t1 = torch.zeros(batch, dtype=torch.int64, device=dev)
    ordt = None
    if order is not None:
        ordt = torch.as_tensor(order, dtype=torch.int32, device=dev)
    _h().posv_mixed_vbatched(batch, nmax, ns, Ap, lda, Bp, ldb, Xp, ldx, nrhs, res, order=ordt, t_start=t0,
                             t_end=t1, params=params, device=dev)
    return Xs, decode_results(res), t0, t1


class SolveFn(torch.autograd.Function):
    """Differentiable x = A^{-1} b through the library's factors.

    forward: getrf + getrs (precision "fp64") or the FP32 factorization with FP64
    refinement ("fp32"); the factors are kept for the backward.
    backward: bbar = A^{-T} xbar from the stored factors (getrs with op T, refined
    in FP64 for "fp32"), Abar = -bbar x^T (outer-product kernel)."""

    @staticmethod
    def forward(ctx, A, b, precision="fp64"):
        vec = b.dim() == A.dim() - 1
        Bm = b.unsqueeze(-1) if vec else b
        Bc = colmajor(Bm.detach())
        Ac = colmajor(A.detach())
        if precision == "fp64":
            LU, ipiv, info = getrf(Ac)
            X = getrs(LU, ipiv, Bc)
            ctx.save_for_backward(LU, ipiv, X)
        else:
            n = A.shape[-1]
            batch = A.shape[0] if A.dim() == 3 else 1
            X = colmajor(torch.zeros_like(Bc))
            LUlo = torch.empty((batch, n * n) if A.dim() == 3 else (n * n,), dtype=torch.float32, device=A.device)
            ipiv = torch.zeros((batch, n) if A.dim() == 3 else (n,), dtype=torch.int32, device=A.device)
            res = torch.zeros(batch * cds.IR_RESULT_BYTES, dtype=torch.uint8, device=A.device)
            _h().gesv_mixed(Ac, Bc, X, LUlo, ipiv, res, precision=precision)
            ctx.save_for_backward(Ac, LUlo, ipiv, X)
        ctx.precision = precision
        ctx.vec = vec
        out = X
        return out.squeeze(-1) if vec else out

    @staticmethod
    def backward(ctx, gx):
        G = gx.unsqueeze(-1) if ctx.vec else gx
        Gc = colmajor(G.contiguous().to(torch.float64))
        if ctx.precision == "fp64":
            LU, ipiv, X = ctx.saved_tensors
            Bbar = getrs(LU, ipiv, Gc, trans=True)
        else:
            Ac, LUlo, ipiv, X = ctx.saved_tensors
            Bbar = colmajor(torch.zeros_like(Gc))
            batch = Ac.shape[0] if Ac.dim() == 3 else 1
            res = torch.zeros(batch * cds.IR_RESULT_BYTES, dtype=torch.uint8, device=Ac.device)
            _h().getrs_mixed(Ac, LUlo, ipiv, Gc, Bbar, res, trans=True)
        n = X.shape[-2]
        Abar = colmajor(torch.empty(X.shape[:-2] + (n, n), dtype=torch.float64, device=X.device))
        _h().outer(Bbar, X, Abar, alpha=-1.0)
        gb = Bbar.squeeze(-1) if ctx.vec else Bbar
        return Abar, gb, None


def solve_ad(A, b, precision="fp64"):
    return SolveFn.apply(A, b, precision)
