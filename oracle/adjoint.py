"""Gradients of a loss of the Stokes solution with respect to the body force
and to a per-element viscosity.

Oracle (test infrastructure only).  For A x = b(f) with b_F = (M f)_F (the
load of the nodal force f on the free velocity DoFs), x normalised to zero
plain-mean pressure (x_hat = P x) and a loss L(x_hat), the chain rule gives

    dL/df = (db/df)^T A^+ P dL/dx_hat,   (db/df)^T = M R_F^T,

A being symmetric.  For a per-element viscosity nu_e the operator depends
on nu_e only through the velocity blocks nu_e L_e (homogeneous Dirichlet
data, so b does not), and with lambda = A^+ P dL/dx_hat

    dL/dnu_e = -lambda_e^T (dA/dnu_e) x = -sum_c lambda_{c,e}^T L_e x_{c,e}

over the free velocity DoFs of element e (L_e the element Laplacian per
unit viscosity).  The solves are dense solves of the bordered system (tiny
meshes only); a direct restatement of the definitions, no multigrid.
``iterative_gradients`` forms the same gradients from forward and adjoint
solves by the oracle's own multigrid-preconditioned FGMRES, for meshes too
large for dense solves; a CPU test checks it against the dense path.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from stokes_inputs import grid_sizes, velocity_dirichlet_mask
from .fem import assemble_q2_mass, element_dof_maps, element_matrices, stokes_system


def _bordered_solve(A, rhs, off_p):
    n = A.shape[0]
    c = np.zeros(n)
    c[off_p:] = 1.0
    K = np.zeros((n + 1, n + 1))
    K[:n, :n] = A.toarray()
    K[:n, n] = c
    K[n, :n] = c
    return sla.solve(K, np.concatenate([rhs, [0.0]]))[:n]


def project_pressure(N, x):
    off_p = grid_sizes(N).off_p
    y = x.copy()
    y[off_p:] -= y[off_p:].mean()
    return y


def solve(N, f, g=None, nu=1.0):  # nu: scalar or N*N per-element values
    """x_hat(f): the solution with zero plain-mean pressure."""
    A, b, _, _ = stokes_system(N, nu, f_nodal=f, g_nodal=g)
    x = _bordered_solve(A, b, grid_sizes(N).off_p)
    return project_pressure(N, x)


def adjoint_state(N, dL_dx, nu=1.0):
    gs = grid_sizes(N)
    A, _, _, _ = stokes_system(N, nu)
    return _bordered_solve(A, project_pressure(N, dL_dx), gs.off_p)


def force_gradient(N, dL_dx, nu=1.0):
    """dL/df (shape (2, (2N+1)^2)) from dL/dx_hat."""
    return force_gradient_from_adjoint(N, adjoint_state(N, dL_dx, nu))


def force_gradient_from_adjoint(N, lam):
    """dL/df = M R_F^T lambda_u for the adjoint state lambda."""
    gs = grid_sizes(N)
    free = ~velocity_dirichlet_mask(N)[:gs.off_p]
    lu = np.where(free, lam[:gs.off_p], 0.0).reshape(2, -1)
    M = assemble_q2_mass(N)
    return np.stack([M @ lu[0], M @ lu[1]])


def viscosity_gradient(N, dL_dx, x, nu):
    """dL/dnu_e (N*N values, index ey*N + ex) from dL/dx_hat at the solution
    x of the per-element viscosity nu."""
    return viscosity_gradient_from_adjoint(N, adjoint_state(N, dL_dx, nu), x)


def viscosity_gradient_from_adjoint(N, lam, x):
    """dL/dnu_e = -sum_c lambda_{c,e}^T L_e x_{c,e} over the free velocity
    DoFs of each element, for the adjoint state lambda and the solution x."""
    gs = grid_sizes(N)
    free = ~velocity_dirichlet_mask(N)[:gs.off_p]
    lu = np.where(free, lam[:gs.off_p], 0.0).reshape(2, -1)
    xu = np.where(free, x[:gs.off_p], 0.0).reshape(2, -1)
    E = element_matrices(1.0 / N)["L"]
    q2, _ = element_dof_maps(N)
    g = np.zeros(N * N)
    for c in range(2):
        g -= np.einsum("ei,ij,ej->e", lu[c][q2], E, xu[c][q2])
    return g


def iterative_gradients(N, levels, f, dL_dx_of, nu, rtol=1e-10, max_iters=80):
    """The same gradients on meshes too large for the dense solves: the
    forward and adjoint systems solved by the oracle's multigrid-
    preconditioned FGMRES (oracle.multigrid, oracle.fgmres) to ``rtol``.
    ``dL_dx_of(x_hat)`` returns dL/dx_hat.  Returns (x_hat, dL/df, dL/dnu)
    and the two FGMRES results."""
    from .fgmres import fgmres
    from .multigrid import Hierarchy
    H = Hierarchy(N, levels, nu=nu)
    A, b, _, xl = stokes_system(N, nu, f_nodal=f)
    fw = fgmres(A, b, xl, H.vcycle, rtol=rtol, restart=30, max_iters=max_iters)
    x_hat = project_pressure(N, fw.x)
    rhs = project_pressure(N, dL_dx_of(x_hat))
    dmask = velocity_dirichlet_mask(N)
    lam0 = np.where(dmask, rhs, 0.0)
    aw = fgmres(A, rhs, lam0, H.vcycle, rtol=rtol, restart=30, max_iters=max_iters)
    lam = aw.x
    return (x_hat, force_gradient_from_adjoint(N, lam),
            viscosity_gradient_from_adjoint(N, lam, x_hat), fw, aw)
