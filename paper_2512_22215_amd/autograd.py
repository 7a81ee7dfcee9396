"""Differentiable LDU solve: x = A(diag, upper, lower)^-1 b as a torch Function.

Backward is the adjoint method: lambda = A^-T (dL/dx) solved on the
transposed coefficients by the same GPU solver, then dL/db = lambda,
dL/ddiag = -lambda o x, dL/dupper_f = -lambda[own] x[nb],
dL/dlower_f = -lambda[nb] x[own], all computed by the HIP library.
"""
from __future__ import annotations

import torch

from .ldu import LduMatrix


class LduSolve(torch.autograd.Function):
    """LduSolve.apply(diag, upper, lower, b, matrix, method, opts) -> x.

    matrix: an LduMatrix holding the addressing; its coefficients are replaced
    by (diag, upper, lower) before the forward solve.  method: "pcg", "gamg"
    or "pbicg" (non-symmetric A); opts: dict of solver options used for both
    solves.
    """

    @staticmethod
    def forward(ctx, diag, upper, lower, b, matrix: LduMatrix, method="pcg", opts=None):
        opts = dict(opts or {})
        matrix.set_coeffs(diag.detach(), upper.detach(), lower.detach())
        solve = {"gamg": matrix.gamg, "pbicg": matrix.pbicg, "pcg": matrix.pcg}[method]
        x, st = solve(b.detach(), **opts)
        ctx.matrix, ctx.method, ctx.opts = matrix, method, opts
        ctx.save_for_backward(x)
        ctx.forward_stats = st
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        m = ctx.matrix
        lam, _ = m.adjoint(gx.detach().to(torch.float64).contiguous(), solver=ctx.method,
                           **ctx.opts)
        gd, gu, gl = m.coeff_grad(lam, x)
        return gd, gu, gl, lam, None, None, None


def ldu_solve(diag, upper, lower, b, matrix: LduMatrix, method="pcg", **opts):
    return LduSolve.apply(diag, upper, lower, b, matrix, method, opts)
