"""Seeded synthetic inputs for the structured Q2-Q1 Stokes problem.

This package holds problem data only: grid geometry, the manufactured
solutions and their forcing terms, seeded random fields and vectors.  It
holds none of the solver's arithmetic (no assembly, no relaxation, no
multigrid, no Krylov method), so that both the CPU oracle and the GPU
library's callers can draw identical inputs from it without sharing any of
the method's code.
"""

from .fields import (  # noqa: F401
    GridSizes,
    grid_sizes,
    q2_coords,
    q1_coords,
    q2_boundary_mask,
    velocity_dirichlet_mask,
    MANUFACTURED,
    manufactured_nodal_force,
    manufactured_boundary_values,
    manufactured_exact_vector,
    lid_boundary_values,
    gaussian_random_field,
    uniform_vector,
    dirichlet_consistent_pair,
    log_viscosity_field,
)
