"""Differentiable Stokes solve with respect to the body force.

``stokes_solve(f, solver, g=None)`` returns the velocity-pressure solution x
(pressure shifted to zero mean) of A x = b(f, g), where b is the load of the
nodal body force f (vkmg_assemble_rhs) and A the Dirichlet-eliminated Q2-Q1
operator, solved by the library's V-cycle-preconditioned FGMRES.  The
backward pass solves the adjoint system with the same solver (A is
symmetric: A^T = A) and maps the adjoint state back through the transpose
of the force-to-load map:

    dL/df = M R_F^T lambda_u,   A lambda = P (dL/dx),

with R_F the restriction to free velocity DoFs and P the pressure-mean
projection (its own transpose).  Every step runs in the library; PyTorch
only supplies the tensors.
"""

from __future__ import annotations

import torch

from ._vkmg import VkmgError


class _StokesSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, solver, g, rtol, restart, max_iters):
        b = solver.assemble_rhs(f.detach().contiguous(), g)
        # initial guess: the Dirichlet lifting (boundary rows of b)
        x = torch.where(solver.dirichlet_mask(), b, torch.zeros_like(b))
        info = solver.fgmres_solve(b, x, rtol=rtol, restart=restart, max_iters=max_iters)
        _require_converged(info, "forward solve")
        solver.remove_pressure_mean(x)
        ctx.solver = solver
        ctx.opts = (rtol, restart, max_iters)
        return x

    @staticmethod
    def backward(ctx, gx):
        solver = ctx.solver
        rtol, restart, max_iters = ctx.opts
        rhs = gx.detach().to(torch.float64).contiguous().clone()
        solver.remove_pressure_mean(rhs)
        # the adjoint's Dirichlet rows are identity rows decoupled from the
        # free DoFs: start from their exact values
        lam = torch.where(solver.dirichlet_mask(), rhs, torch.zeros_like(rhs))
        info = solver.fgmres_solve(rhs, lam, rtol=rtol, restart=restart, max_iters=max_iters)
        _require_converged(info, "adjoint solve")
        grad_f = solver.assemble_rhs_adjoint(lam)
        return grad_f, None, None, None, None, None


def _require_converged(info, where):
    infos = info if isinstance(info, list) else [info]
    for i in infos:
        if i["status_name"] != "VKMG_OK":
            raise VkmgError(6, where, f"FGMRES did not converge: {i}")


def stokes_solve(f, solver, g=None, rtol: float = 1e-10, restart: int = 30,
                 max_iters: int = 500):
    """x(f) for nodal body force f (2 (2N+1)^2 doubles per right-hand side,
    [f_x | f_y]) and Dirichlet data g (same size, or None); differentiable
    with respect to f."""
    return _StokesSolve.apply(f, solver, g, rtol, restart, max_iters)
