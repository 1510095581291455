"""Plain FP64 CPU oracle for the Vanka-multigrid-preconditioned FGMRES solver
of the structured Q2-Q1 Stokes discretisation.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or
calls this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the HIP path: it assembles the
sparse saddle-point matrix from the finite-element definitions, extracts the
Vanka patch blocks from that matrix by brute force, and runs the same
multigrid V-cycle and FGMRES step by step with NumPy/SciPy in float64.

Modules (each function cites the passage of the paper it follows):
  fem        element integrals, global assembly, Dirichlet elimination,
             right-hand sides, discretisation errors
  transfer   finite-element interpolation between nested grids
  vanka      patches, patch inverses, additive Vanka sweep
  multigrid  level hierarchy, coarse bordered solve, V-cycle
  fgmres     restarted flexible GMRES

Parity status: every function is pinned by a CPU test against the
mathematics (closed forms, exact polynomial reproduction, dense direct
solves, spectral properties, brute-force least squares); FGMRES iteration
counts at the benchmark sizes are "parity unpinned" by the paper, which
prints none.
"""

from . import fem, transfer, vanka, multigrid, fgmres  # noqa: F401
