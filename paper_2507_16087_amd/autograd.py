"""Differentiable solve: pressure field as a function of (c, rho, alpha).

``CBSSolve.apply(c, rho, alpha, s_p, spec)`` runs the forward solve
A(m) xi = s_hat(m) on the GPU and returns the complex pressure p.  Its
backward pass is the adjoint-state method on the adjoint operator of the
paper (Sec. 2.3: negated differential part, conjugated diagonal): given the
incoming gradient g (torch's convention for complex outputs, so that
dL = Re <g, dp>), it solves A^H lambda = (0, g) with the same iteration run
on the adjoint, then the gradient kernel forms

    dL/dm(x) = Re sum_rows conj(lambda_row) [d s_hat_row/dm(x) - dD_row/dm(x) xi_row]

for m in {c, rho, alpha}.  Both solves use the precision in ``spec``.
"""
from __future__ import annotations

import dataclasses

import torch

from . import solver


@dataclasses.dataclass(frozen=True)
class SolveSpec:
    shape: tuple
    dx: float
    omega: float
    pml: int = 16
    prec: str = "fp32_refined"
    tol: float = 1e-8
    max_iter: int = 200000
    inner_tol: float = 0.0


class CBSSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, rho, alpha, s_p, spec: SolveSpec):
        for t in (c, rho, alpha):
            if not (t.is_cuda and t.dtype == torch.float64):
                raise ValueError("c, rho, alpha must be float64 CUDA tensors")
        m = solver.Medium(spec.shape, spec.dx, spec.omega, c.detach(), rho.detach(), alpha.detach(),
                          pml=spec.pml)
        sp = s_p.detach().to(torch.complex128).contiguous().reshape(-1)
        p, u, info = solver.solve(m, sp, tol=spec.tol, max_iter=spec.max_iter, prec=spec.prec,
                                  inner_tol=spec.inner_tol, want_u=True)
        if not info["converged"]:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.m, ctx.spec = m, spec
        ctx.save_for_backward(sp, p, u)
        return p

    @staticmethod
    def backward(ctx, grad_p):
        sp, p, u = ctx.saved_tensors
        m, spec = ctx.m, ctx.spec
        g = grad_p.detach().to(torch.complex128).contiguous().reshape(-1)
        lp, lu, info = solver.solve(m, g, tol=spec.tol, max_iter=spec.max_iter, prec=spec.prec,
                                    inner_tol=spec.inner_tol, equation_rhs=True, adjoint=True,
                                    want_u=True)
        if not info["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        gc, grho, galpha = solver.gradient(m, sp, None, p, u, lp, lu)
        return gc, grho, galpha, None, None


def pressure(c, rho, alpha, s_p, spec: SolveSpec):
    """Differentiable pressure field p(c, rho, alpha) for source s_p."""
    return CBSSolve.apply(c, rho, alpha, s_p, spec)
