"""Gradient of a loss of the Stokes solution with respect to the body force.

Oracle (test infrastructure only).  For A x = b(f) with b_F = (M f)_F (the
load of the nodal force f on the free velocity DoFs), x normalised to zero
plain-mean pressure (x_hat = P x) and a loss L(x_hat), the chain rule gives

    dL/df = (db/df)^T A^+ P dL/dx_hat,   (db/df)^T = M R_F^T,

A being symmetric.  The solves are dense least-squares solves of the
bordered system (tiny meshes only); a direct restatement of the definition,
no multigrid.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from stokes_inputs import grid_sizes, velocity_dirichlet_mask
from .fem import assemble_q2_mass, stokes_system


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


def solve(N, f, g=None, nu=1.0):
    """x_hat(f): the solution with zero plain-mean pressure."""
    A, b, _, _ = stokes_system(N, nu, f_nodal=f, g_nodal=g)
    x = _bordered_solve(A, b, grid_sizes(N).off_p)
    return project_pressure(N, x)


def force_gradient(N, dL_dx, nu=1.0):
    """dL/df (shape (2, (2N+1)^2)) from dL/dx_hat."""
    gs = grid_sizes(N)
    A, _, _, _ = stokes_system(N, nu)
    lam = _bordered_solve(A, project_pressure(N, dL_dx), gs.off_p)
    free = ~velocity_dirichlet_mask(N)[:gs.off_p]
    lu = np.where(free, lam[:gs.off_p], 0.0).reshape(2, -1)
    M = assemble_q2_mass(N)
    return np.stack([M @ lu[0], M @ lu[1]])
