"""Differentiable Stokes solve with respect to the body force and a
per-element viscosity.

``stokes_solve(f, solver, g=None, nu=None)`` returns the velocity-pressure
solution x (pressure shifted to zero mean) of A(nu) x = b(f, g), where b is
the load of the nodal body force f (vkmg_assemble_rhs) and A the
Dirichlet-eliminated Q2-Q1 operator, solved by the library's
V-cycle-preconditioned FGMRES.  The backward pass solves the adjoint system
with the same solver (A is symmetric: A^T = A) and maps the adjoint state
back:

    A lambda = P dL/dx,   dL/df = M R_F^T lambda_u,
    dL/dnu_e = -sum_c lambda_{c,e}^T L_e x_{c,e},

with R_F the restriction to free velocity DoFs, P the pressure-mean
projection (its own transpose) and L_e the element Laplacian per unit
viscosity.  `nu` (N*N values, index ey*N + ex) must be the field the solver
was set up with (VkmgSolver(..., nu_elem=...)); it is an input only so that
autograd can route its gradient.  Every step runs in the library; PyTorch
only supplies the tensors.
"""

from __future__ import annotations

import torch

from ._vkmg import VkmgError


class _StokesSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, nu, solver, g, rtol, restart, max_iters):
        b = solver.assemble_rhs(f.detach().contiguous(), g)
        # initial guess: the Dirichlet lifting (boundary rows of b)
        x = solver.dirichlet_lift(b)
        info = solver.fgmres_solve(b, x, rtol=rtol, restart=restart, max_iters=max_iters)
        _require_converged(info, "forward solve")
        solver.remove_pressure_mean(x)
        ctx.solver = solver
        ctx.opts = (rtol, restart, max_iters)
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        solver = ctx.solver
        (x,) = ctx.saved_tensors
        rtol, restart, max_iters = ctx.opts
        rhs = gx.detach().to(torch.float64).contiguous().clone()
        solver.remove_pressure_mean(rhs)
        # the adjoint's Dirichlet rows are identity rows decoupled from the
        # free DoFs: start from their exact values
        lam = solver.dirichlet_lift(rhs)
        info = solver.fgmres_solve(rhs, lam, rtol=rtol, restart=restart, max_iters=max_iters)
        _require_converged(info, "adjoint solve")
        grad_f = solver.assemble_rhs_adjoint(lam) if ctx.needs_input_grad[0] else None
        grad_nu = solver.viscosity_gradient(lam, x) if ctx.needs_input_grad[1] else None
        return grad_f, grad_nu, None, None, None, None, None


def _require_converged(info, where):
    infos = info if isinstance(info, list) else [info]
    for i in infos:
        if i["status_name"] != "VKMG_OK":
            raise VkmgError(6, where, f"FGMRES did not converge: {i}")


def stokes_solve(f, solver, g=None, nu=None, rtol: float = 1e-10, restart: int = 30,
                 max_iters: int = 500):
    """x(f, nu) for nodal body force f (2 (2N+1)^2 doubles per right-hand
    side, [f_x | f_y]) and Dirichlet data g (same size, or None);
    differentiable with respect to f and, for solvers set up with a
    per-element viscosity, to that viscosity passed as `nu`."""
    if nu is not None:
        solver.check_viscosity(nu)
    else:
        nu = torch.zeros(0, dtype=torch.float64, device=f.device)
    return _StokesSolve.apply(f, nu, solver, g, rtol, restart, max_iters)
