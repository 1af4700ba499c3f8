"""Differentiable solve: x = A^{-1} b as a torch.autograd.Function.

The forward pass builds the nAIR hierarchy of A and solves A x = b; the
backward pass reuses that hierarchy transposed (P^T restricts, R^T
interpolates, block Jacobi uses D^{-T}) to solve A^T ybar = xbar, and returns
dL/db = ybar and dL/dA = -ybar x^T on A's block pattern.
"""
from __future__ import annotations

import torch

from .nair import Hierarchy, Params, NairError, grad_vals


class NairSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, rowptr, colidx, bs, params, rtol, max_iter):
        H = Hierarchy(rowptr, colidx, vals.detach().contiguous(), bs, params)
        x, res = H.solve(b.detach().contiguous(), rtol=rtol, max_iter=max_iter)
        if res.status != "OK":
            raise NairError(3 if res.status == "ENOCONV" else 4, "forward solve", res.status)
        ctx.H = H
        ctx.bs = bs
        ctx.rtol = rtol
        ctx.max_iter = max_iter
        ctx.forward_result = res
        ctx.save_for_backward(x, rowptr, colidx)
        return x

    @staticmethod
    def backward(ctx, xbar):
        x, rowptr, colidx = ctx.saved_tensors
        H = ctx.H
        ybar, res = H.solve_T(xbar.contiguous(), rtol=ctx.rtol, max_iter=ctx.max_iter)
        if res.status != "OK":
            raise NairError(3 if res.status == "ENOCONV" else 4, "adjoint solve", res.status)
        ctx.backward_result = res
        g_vals = grad_vals(rowptr, colidx, ybar, x, ctx.bs) if ctx.needs_input_grad[0] else None
        g_b = ybar if ctx.needs_input_grad[1] else None
        return g_vals, g_b, None, None, None, None, None, None


def solve(vals, b, rowptr, colidx, bs: int, params: Params | None = None, rtol: float = 1e-10,
          max_iter: int = 200):
    """Differentiable x = A^{-1} b for A = BSR(rowptr, colidx, vals) (device tensors)."""
    return NairSolve.apply(vals, b, rowptr, colidx, int(bs), params or Params(), float(rtol), int(max_iter))
