"""Differentiable multigrid solve: u = A(k)^-1 f as a torch.autograd.Function.

Backward by implicit differentiation of A(k) u = f (the loss sees the converged discrete
solution, not the unrolled iteration): with lambda = A^-T dL/du (A is symmetric, so the
adjoint solve reuses the forward hierarchy),
    dL/df = lambda,   dL/dk = -lambda^T (dA/dk) u,
the second evaluated by one fused gradient pass of the library (mg_grad).  With
``recompute=True`` (the default) the forward solution is not kept: backward re-solves
for u from k and f instead of storing any iterate.

``coarsening="galerkin"`` (3D, FP64) solves forward and adjoint with Galerkin coarse operators
(``GalerkinMultigrid``): the same discrete system, so the same gradient up to the solve
tolerance; its hierarchy depends on k, so it and the forward solution are kept until backward.
"""
from __future__ import annotations

import torch

from .galerkin import GalerkinMultigrid
from .solver import Multigrid


class MGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k, f, mg: Multigrid, tol: float, recompute: bool):
        mg.set_coefficients(k)
        u, info = mg.solve(f, mg.zeros(), tol=tol)
        ctx.mg, ctx.tol, ctx.recompute = mg, tol, recompute
        ctx.fwd_info = info
        if recompute:
            ctx.save_for_backward(k, f)
        else:
            ctx.save_for_backward(k, f, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        mg: Multigrid = ctx.mg
        saved = ctx.saved_tensors
        k, f = saved[0], saved[1]
        mg.set_coefficients(k)
        if ctx.recompute:
            u, _ = mg.solve(f, mg.zeros(), tol=ctx.tol)
        else:
            u = saved[2]
        g = grad_u.contiguous().to(torch.float64)
        lam, _ = mg.solve_adjoint(g, mg.zeros(), tol=ctx.tol)
        dk, df = mg.grad(u, lam, want_k=ctx.needs_input_grad[0], want_f=ctx.needs_input_grad[1])
        return dk, df, None, None, None


class MGSolveGalerkin(torch.autograd.Function):
    """MGSolve with Galerkin coarse operators; mg serves the gradient pass only."""

    @staticmethod
    def forward(ctx, k, f, mg: Multigrid, tol: float, levels):
        gm = GalerkinMultigrid(k.contiguous(), levels)
        u, info = gm.solve(f.contiguous(), tol=tol)
        if not info.converged:
            gm.close()
            raise RuntimeError(f"Galerkin solve: relative residual {info.relres:.3e} > {tol:.1e}")
        ctx.gm, ctx.mg, ctx.tol = gm, mg, tol
        ctx.fwd_info = info
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        gm: GalerkinMultigrid = ctx.gm
        (u,) = ctx.saved_tensors
        lam, info = gm.solve(grad_u.contiguous().to(torch.float64), tol=ctx.tol)
        gm.close()
        if not info.converged:
            raise RuntimeError(f"Galerkin adjoint solve: relative residual {info.relres:.3e} > {ctx.tol:.1e}")
        dk, df = ctx.mg.grad(u, lam, want_k=ctx.needs_input_grad[0], want_f=ctx.needs_input_grad[1])
        return dk, df, None, None, None


def solve(k: torch.Tensor, f: torch.Tensor, mg: Multigrid | None = None, tol: float = 1e-10,
          precision: str = "f64", levels: int | None = None, recompute: bool = True,
          coarsening: str = "rediscretise"):
    """u solving -div(k grad u) = f (zero Dirichlet data), differentiable in k and f.
    coarsening: "rediscretise" (the coefficient hierarchy of Multigrid) or "galerkin"."""
    if coarsening == "galerkin":
        if f.dim() != 3 or precision != "f64":
            raise ValueError("Galerkin coarsening is 3D and FP64")
        if mg is None:  # the gradient pass needs no coefficients
            mg = Multigrid(3, f.shape[0], levels=levels, device=f.device)
        return MGSolveGalerkin.apply(k, f, mg, tol, levels)
    if coarsening != "rediscretise":
        raise ValueError(f"coarsening must be 'rediscretise' or 'galerkin', got {coarsening!r}")
    if mg is None:
        mg = Multigrid(f.dim(), f.shape[0], levels=levels, precision=precision, variable=True,
                       device=f.device)
    return MGSolve.apply(k, f, mg, tol, recompute)
