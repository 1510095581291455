"""Host paths of the C ABI, for the sanitizer build (no GPU).

    python tests/sanitize_driver.py LIBRARY

Loads LIBRARY (normally _build/sanitize/libvkmg_sanitized.so, with the
sanitizer runtime preloaded by the caller) and runs every entry point's
host-side code: option and argument validation, NULL handling, the host
patch matrices of all 25 classes with their inverses, and complete
vkmg_setup / vkmg_setup_viscosity host work (patch matrices, Gauss-Jordan
inverses, symmetry blocks, the bordered coarse inverse, the per-patch
tables on the worker threads), which ends with VKMG_ERR_HIP at the first
device call when no GPU is present.  Prints SANITIZE-DRIVER OK on success.
"""

import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2401_06277_amd import _vkmg  # noqa: E402


def main(path):
    lib = _vkmg.load_library(path)
    Grid = _vkmg.Grid
    ctx = ctypes.c_void_p()

    def setup(N, levels, nu=1.0, **opts):
        o = lib.vkmg_default_options()
        for k, v in opts.items():
            setattr(o, k, v)
        return lib.vkmg_setup(ctypes.byref(Grid(N, N)), levels, nu, ctypes.byref(o), None,
                              ctypes.byref(ctx))

    for s in range(9):
        assert lib.vkmg_status_string(s)
    # validation
    assert lib.vkmg_setup(ctypes.byref(Grid(16, 8)), 3, 1.0, None, None, ctypes.byref(ctx)) == 1
    assert lib.vkmg_setup(None, 3, 1.0, None, None, None) == 1
    for bad in (dict(mg_precision=2), dict(omega=0.0), dict(nu_pre=-1), dict(batch=65),
                dict(relaxation=2), dict(bs_jacobi_sweeps=0), dict(bs_t=-1.0)):
        assert setup(16, 3, **bad) == 1, bad
        assert lib.vkmg_last_error()
    assert setup(20, 4) == 1 and setup(256, 2) == 2 and setup(16, 3, nu=float("nan")) == 1
    # every context entry point rejects a NULL context
    P = None
    assert lib.vkmg_residual(P, P, P, P, P) == 1
    assert lib.vkmg_apply(P, P, P, P) == 1
    assert lib.vkmg_vanka_sweep(P, 1, P, P, P) == 1
    assert lib.vkmg_vanka_update(P, 1, P, P, P) == 1
    assert lib.vkmg_relax(P, 1, P, P, P) == 1
    assert lib.vkmg_restrict(P, 1, P, P, P) == 1
    assert lib.vkmg_prolong_add(P, 1, P, P, P) == 1
    assert lib.vkmg_coarse_solve(P, P, P, P) == 1
    assert lib.vkmg_vcycle(P, P, P, P) == 1
    assert lib.vkmg_fgmres_solve(P, P, P, 1e-8, 30, 10, None, P) == 1
    if hasattr(lib, "vkmg_fgmres_solve_noalloc"):
        assert lib.vkmg_fgmres_solve_noalloc(P, P, P, 1e-8, 30, 10, None, P) == 1
    assert lib.vkmg_set_timing(P, 1) == 1
    lib.vkmg_destroy(None)
    # host patch matrices of every class
    A = np.empty(51 * 51)
    Ai = np.empty(51 * 51)
    W = np.empty(51 * 51)
    pres = np.empty(51, dtype=np.uint8)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    for N in (4, 8, 16, 64):
        for c in range(25):
            st = lib.vkmg_host_patch_matrix(N, 1.5, 0.5, c, ptr(A), ptr(Ai), ptr(W), ptr(pres))
            assert st == 0, (N, c)
            M = A.reshape(51, 51) @ Ai.reshape(51, 51)
            assert np.abs(M - np.eye(51)).max() < 1e-11
    assert lib.vkmg_host_patch_matrix(8, 1.0, 0.5, 25, ptr(A), P, P, P) == 1
    # complete host setup work (stops at the first device call without a GPU)
    for N, L, opts in ((16, 3, {}), (64, 4, dict(mg_precision=1)), (32, 3, dict(batch=2)),
                       (32, 3, dict(relaxation=1)), (128, 5, dict(interior_apply=1))):
        st = setup(N, L, **opts)
        assert st in (0, 4), (N, L, opts, st, lib.vkmg_last_error())
        if st == 0:
            lib.vkmg_destroy(ctx)
    nu = np.exp(np.random.default_rng(7).uniform(-1.0, 1.0, 32 * 32))
    st = lib.vkmg_setup_viscosity(ctypes.byref(Grid(32, 32)), 3, ptr(nu), None, None,
                                  ctypes.byref(ctx))
    assert st in (0, 4), (st, lib.vkmg_last_error())
    if st == 0:
        lib.vkmg_destroy(ctx)
    print("SANITIZE-DRIVER OK", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
