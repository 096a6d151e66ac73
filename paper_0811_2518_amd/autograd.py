"""torch.autograd.Function around gabp_solve / gabp_backward.

Forward: x = A^-1 b by GaBP.  Backward: lambda = A^-1 dL/dx by a second GaBP
solve against the symmetric A, dL/db = lambda and dL/dA on the stored pattern
(-(lambda_i x_j + lambda_j x_i) off the diagonal, mirror entries tied;
-lambda_i x_i on it), both computed by the library.
"""
from __future__ import annotations

import torch


class GaBPSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, vals, b, tol, max_iter):
        x, info = solver.solve(b, tol=tol, max_iter=max_iter)
        ctx.solver = solver
        ctx.tol, ctx.max_iter = tol, max_iter
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        (x,) = ctx.saved_tensors
        gb, gv, _ = ctx.solver.backward(x, grad_x.contiguous(), tol=ctx.tol, max_iter=ctx.max_iter,
                                        grad_vals=ctx.needs_input_grad[1])
        return None, gv, gb, None, None


def gabp_solve(solver, vals, b, tol=1e-12, max_iter=5000):
    """x = A^-1 b with gradients to ``vals`` (the CSR values the solver was built from) and ``b``."""
    return GaBPSolve.apply(solver, vals, b, tol, max_iter)
