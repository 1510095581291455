"""vkmg: Vanka-multigrid preconditioned FGMRES for the structured-grid
Q2-Q1 Stokes discretisation on AMD Instinct MI355X (gfx950).

The numerical work runs in the HIP library ``libvkmg.so`` (C ABI declared in
include/vkmg.h); this package is its Python binding.
"""

from ._vkmg import (  # noqa: F401
    EXPORTED,
    FP32,
    FP64,
    KERNEL_COARSE,
    KERNEL_KRYLOV,
    KERNEL_RESIDUAL,
    KERNEL_TRANSFER,
    KERNEL_VANKA,
    KERNEL_VANKA_TILE,
    LIB_PATH,
    STATUS,
    VkmgError,
    VkmgSolver,
    default_options,
    host_patch_matrix,
    load_library,
)
