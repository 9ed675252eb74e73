"""torch.autograd.Function around the solve and its hand-written adjoint.

Forward: x = A^-1 b with A assembled from (diag, upper, lower) on a Mesh.
Backward: one more solve, A^T lambda = dL/dx (A is symmetric for CG, so the
same solver), then dL/db = lambda and dL/dA on the sparsity pattern
(dL/ddiag = -lambda*x, dL/dupper[f] = -lambda[owner] x[neighbour],
dL/dlower[f] = -lambda[neighbour] x[owner]), all in libfvpcg.so.
Chaining to face conductivities is left to differentiable torch assembly in
the caller.
"""
from __future__ import annotations

import torch


class FVSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, diag, upper, lower, b, mesh, opts=None):
        from . import Matrix, solve

        opts = dict(opts or {})
        tol = opts.get("tol", 1e-10)
        maxit = opts.get("maxit", 20000)
        method = opts.get("method", "pipecg")
        precond = opts.get("precond", "jacobi")
        sym = lower is None
        A = Matrix(mesh, diag.detach().contiguous(), upper.detach().contiguous(),
                   None if sym else lower.detach().contiguous())
        x, st = solve(A, b.detach().contiguous(), tol=tol, maxit=maxit, method=method, precond=precond)
        ctx.A = A
        ctx.sym = sym
        ctx.opts = (opts.get("adjoint_tol", tol), maxit, method, precond)
        ctx.stats = st
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        from . import solve_backward

        (x,) = ctx.saved_tensors
        tol, maxit, method, precond = ctx.opts
        want = ("b", "diag", "upper") if ctx.sym else ("b", "diag", "upper", "lower")
        g, _ = solve_backward(ctx.A, x, gx.contiguous(), want=want, tol=tol, maxit=maxit, method=method,
                              precond=precond)
        return g["diag"], g["upper"], (None if ctx.sym else g["lower"]), g["b"], None, None


def fv_solve(diag, upper, lower, b, mesh, **opts):
    """Differentiable x = A(diag, upper, lower)^-1 b on `mesh`."""
    return FVSolve.apply(diag, upper, lower, b, mesh, opts)
