"""torch.autograd.Function around the GPU solver.

Forward: x = A^{-1} b with the solver's IC(0) factor, mode (plain, deflated,
subspace correction) and precision.  Backward: for the loss gradient g = dL/dx
the adjoint solve lambda = A^{-T} g = A^{-1} g (A is symmetric) reuses the same
factor and auxiliary space W; then dL/db = lambda and, for every stored entry
(i, j) of A, dL/da_ij = -lambda_i x_j (the partial derivative of a general
matrix entry; esd_grad_values).  Both the solve and the gradient run in the
HIP library.

`vals` is the float64 CUDA tensor of the stored values in the caller's CSR
order; it must hold the values the solver was set up (or last updated) with —
it is the leaf the gradient is returned for, the solver does not re-read it.
"""
from __future__ import annotations

import torch

from . import esd


class ESDSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, solver, mode=esd.PLAIN, tol=1e-8, maxit=20000, flags=0):
        if vals.numel() != solver.nnz:
            raise ValueError("vals must hold the %d stored values" % solver.nnz)
        x, info = solver.solve(b.detach(), tol=tol, maxit=maxit, mode=mode, flags=flags)
        if not info["converged"]:
            raise RuntimeError("forward solve did not converge: %s" % info)
        ctx.solver = solver
        ctx.args = (mode, tol, maxit, flags)
        ctx.info = info
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        solver = ctx.solver
        mode, tol, maxit, flags = ctx.args
        lam, info = solver.solve(gx.detach().contiguous(), tol=tol, maxit=maxit, mode=mode, flags=flags)
        if not info["converged"]:
            raise RuntimeError("adjoint solve did not converge: %s" % info)
        gvals = solver.grad_values(lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gvals, gb, None, None, None, None, None


def solve(vals, b, solver, mode=esd.PLAIN, tol=1e-8, maxit=20000, flags=0):
    """Differentiable x = A^{-1} b (see ESDSolve)."""
    return ESDSolve.apply(vals, b, solver, mode, tol, maxit, flags)
