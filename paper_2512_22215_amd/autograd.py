"""Differentiable LDU solve: x = A(diag, upper, lower)^-1 b as a torch Function.

Backward is the adjoint method: lambda = A^-T (dL/dx) solved on the
transposed coefficients by the same GPU solver, then dL/db = lambda,
dL/ddiag = -lambda o x, dL/dupper_f = -lambda[own] x[nb],
dL/dlower_f = -lambda[nb] x[own], all computed by the HIP library.
"""
from __future__ import annotations

import torch

from .ldu import LDU_NOT_CONVERGED, LduError, LduMatrix


class LduSolve(torch.autograd.Function):
    """LduSolve.apply(diag, upper, lower, b, matrix, method, opts) -> x.

    matrix: an LduMatrix holding the addressing; its coefficients are replaced
    by (diag, upper, lower) before the forward solve.  method: "pcg", "gamg"
    or "pbicg" (non-symmetric A); opts: dict of solver options used for both
    solves.  Several solves may share one matrix before their backward
    passes: a backward whose coefficients are no longer the matrix's puts its
    own back first.  A forward or adjoint solve that stops above its
    tolerance raises LduError (code LDU_NOT_CONVERGED).
    """

    @staticmethod
    def forward(ctx, diag, upper, lower, b, matrix: LduMatrix, method="pcg", opts=None):
        opts = dict(opts or {})
        coeffs = (diag.detach(), upper.detach(), lower.detach())
        matrix.set_coeffs(*coeffs)
        solve = {"gamg": matrix.gamg, "pbicg": matrix.pbicg, "pcg": matrix.pcg}[method]
        x, st = solve(b.detach(), **opts)
        if not st.converged:
            raise LduError(LDU_NOT_CONVERGED,
                           f"forward {method} solve stopped at relative residual "
                           f"{st.final_residual:.3e} after {st.iterations} iterations")
        ctx.matrix, ctx.method, ctx.opts = matrix, method, opts
        ctx.version = matrix.coeff_version
        ctx.save_for_backward(x, *coeffs)
        ctx.forward_stats = st
        return x

    @staticmethod
    def backward(ctx, gx):
        x, diag, upper, lower = ctx.saved_tensors
        m = ctx.matrix
        if m.coeff_version != ctx.version:
            # another solve replaced the coefficients since this forward
            m.set_coeffs(diag, upper, lower)
            ctx.version = m.coeff_version
        lam, st = m.adjoint(gx.detach().to(torch.float64).contiguous(), solver=ctx.method,
                            **ctx.opts)
        if not st.converged:
            raise LduError(LDU_NOT_CONVERGED,
                           f"adjoint {ctx.method} solve stopped at relative residual "
                           f"{st.final_residual:.3e} after {st.iterations} iterations")
        gd, gu, gl = m.coeff_grad(lam, x)
        return gd, gu, gl, lam, None, None, None


def ldu_solve(diag, upper, lower, b, matrix: LduMatrix, method="pcg", **opts):
    return LduSolve.apply(diag, upper, lower, b, matrix, method, opts)
