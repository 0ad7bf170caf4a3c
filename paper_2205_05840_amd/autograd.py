"""Differentiable solve u_r = A(alpha)^{-1} b_r as a torch.autograd.Function.

A(alpha) = alpha K + M is symmetric (Sec. 2, eq. def bilinear form), so the adjoint
system uses the same operator and the same V-cycle-preconditioned CG:
    A lambda_r = dL/du_r,   dL/db_r = lambda_r,   dL/dalpha = -sum_r lambda_r^T K u_r,
the last one from the fused curl-curl form kernel (K = dA/dalpha).  Entries outside the
unknowns carry no gradient.
"""
import torch

from .solver import Solver


def _solve_rows(solver, B2, rtol, maxit):
    """Solve every row of B2 [k, vec_len]: all at once when the solver holds k
    right-hand sides, else one row at a time (single right-hand-side solver)."""
    k = B2.shape[0]
    if solver.nrhs == k:
        U, it, _ = solver.solve(B2, rtol, maxit)
        return U, (list(it) if isinstance(it, list) else [it])
    if solver.nrhs != 1:
        raise ValueError(f"the solver holds {solver.nrhs} right-hand sides, got {k}")
    U = torch.zeros_like(B2)
    iters = []
    for r in range(k):
        _, it, _ = solver.solve(B2[r].contiguous(), rtol, maxit, u=U[r])
        iters.append(it)
    return U, iters


class _SolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, B, alpha, solver, rtol, maxit):
        if abs(float(alpha) - solver.alpha) > 1e-14 * max(1.0, abs(solver.alpha)):
            raise ValueError("alpha must equal the solver's alpha (build one solver per alpha)")
        B2 = B.reshape(-1, solver.vec_len)
        U, iters = _solve_rows(solver, B2.contiguous(), rtol, maxit)
        ctx.solver, ctx.rtol, ctx.maxit = solver, rtol, maxit
        ctx.iters = iters
        ctx.save_for_backward(U)
        return U.reshape(B.shape)

    @staticmethod
    def backward(ctx, gU):
        (U,) = ctx.saved_tensors
        S = ctx.solver
        G = (gU.reshape(-1, S.vec_len) * S.unknown_mask()).contiguous()
        Lam, _ = _solve_rows(S, G, ctx.rtol, ctx.maxit)
        galpha = -S.curlcurl_form(Lam, U)
        return (Lam.reshape(gU.shape),
                torch.tensor(galpha, dtype=torch.float64, device=gU.device), None, None, None)


def solve(B, alpha, solver: Solver, rtol=1e-12, maxit=500):
    """U = A(alpha)^{-1} B for stacked right-hand sides B [..., vec_len] (padded layout),
    differentiable with respect to B and alpha (a 0-dim float64 tensor)."""
    if not torch.is_tensor(alpha):
        alpha = torch.tensor(float(alpha), dtype=torch.float64, device=B.device)
    return _SolveFn.apply(B, alpha, solver, rtol, maxit)
