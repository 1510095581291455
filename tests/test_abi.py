"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, validates arguments before touching the GPU, and its host-side setup
(the 25 Vanka patch matrices and their inverses) agrees with the oracle's
brute-force extraction from the assembled matrix."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2401_06277_amd as vk
from oracle import fem, vanka

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "vkmg.h")) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(vkmg_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = vk.load_library()
    decl = declared_symbols()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(decl) == sorted(vk.EXPORTED)



def test_missing_library_fails_loudly(monkeypatch):
    """Without the built HIP library nothing falls back to another path:
    loading it, and constructing a solver, raise."""
    from paper_2401_06277_amd import _vkmg

    real_exists = os.path.exists
    monkeypatch.setattr(_vkmg, "_lib", None)
    monkeypatch.setattr(os.path, "exists",
                        lambda p: False if str(p).endswith("libvkmg.so") else real_exists(p))
    with pytest.raises(RuntimeError, match="not built"):
        _vkmg.load_library()
    with pytest.raises(RuntimeError, match="not built"):
        vk.VkmgSolver(16, 3)

def test_default_options_and_status_strings():
    lib = vk.load_library()
    o = lib.vkmg_default_options()
    assert (o.nu_pre, o.nu_post, o.omega, o.mg_precision, o.interior_apply,
            o.use_graphs, o.batch) == (2, 2, 0.5, 0, 0, 1, 1)
    for s in range(8):
        assert lib.vkmg_status_string(s)


@pytest.mark.parametrize("kwargs,status", [
    (dict(nx=16, ny=8, levels=3, nu=1.0), 1),      # nx != ny
    (dict(nx=16, ny=16, levels=1, nu=1.0), 1),     # too few levels
    (dict(nx=20, ny=20, levels=4, nu=1.0), 1),     # not divisible by 2^(L-1)
    (dict(nx=16, ny=16, levels=5, nu=1.0), 1),     # coarsest 1x1
    (dict(nx=16, ny=16, levels=3, nu=0.0), 1),     # nu must be positive
    (dict(nx=16, ny=16, levels=3, nu=float("nan")), 1),
    (dict(nx=256, ny=256, levels=2, nu=1.0), 2),   # dense coarse solve too large
])
def test_setup_rejects_bad_arguments_before_any_gpu_work(kwargs, status):
    lib = vk.load_library()
    from paper_2401_06277_amd._vkmg import Grid
    ctx = ctypes.c_void_p()
    st = lib.vkmg_setup(ctypes.byref(Grid(kwargs["nx"], kwargs["ny"])), kwargs["levels"],
                        kwargs["nu"], None, None, ctypes.byref(ctx))
    assert st == status
    assert lib.vkmg_last_error()
    assert not ctx.value


@pytest.mark.parametrize("field,value", [("mg_precision", 2), ("interior_apply", 2),
                                         ("omega", 0.0), ("nu_pre", -1), ("use_graphs", 2),
                                         ("batch", 0), ("batch", 65)])
def test_setup_rejects_bad_options(field, value):
    lib = vk.load_library()
    from paper_2401_06277_amd._vkmg import Grid
    o = lib.vkmg_default_options()
    setattr(o, field, value)
    ctx = ctypes.c_void_p()
    st = lib.vkmg_setup(ctypes.byref(Grid(16, 16)), 3, 1.0, ctypes.byref(o), None,
                        ctypes.byref(ctx))
    assert st == 1 and not ctx.value
    assert lib.vkmg_last_error()


def test_null_arguments_are_rejected():
    lib = vk.load_library()
    assert lib.vkmg_residual(None, None, None, None, None) == 1
    assert lib.vkmg_vcycle(None, None, None, None) == 1
    assert lib.vkmg_fgmres_solve(None, None, None, 1e-8, 30, 10, None, None) == 1
    assert lib.vkmg_setup(None, 3, 1.0, None, None, None) == 1
    lib.vkmg_destroy(None)  # NULL-safe


@pytest.mark.parametrize("N,nu", [(4, 1.0), (8, 1.0), (16, 2.5)])
def test_host_patch_matrices_match_oracle_extraction(N, nu):
    A_full = fem.stokes_system(N, nu)[0]
    idx = vanka.patch_dofs(N)
    cls = vanka.patch_classes(N)
    for c in range(25):
        k = np.nonzero(cls == c)[0][0]
        A, Ai, W, pres = vk.host_patch_matrix(N, nu, 0.5, c)
        assert np.array_equal(pres, idx[k] >= 0)
        S = np.nonzero(pres)[0]
        Ak = vanka.extract_patch_matrix(A_full, idx[k])
        assert np.abs(A[np.ix_(S, S)] - Ak).max() <= 1e-14 * np.abs(Ak).max()
        assert np.abs(A @ Ai - np.eye(51)).max() < 1e-12
        # the weighted inverse is the oracle's W_i A_i^{-1}
        w = vanka.vanka_weights(N, fem.stokes_system(N, nu)[2], 0.5)
        inv_o = np.linalg.inv(Ak)
        Wo = w[idx[k][S]][:, None] * inv_o
        assert np.abs(W[np.ix_(S, S)] - Wo).max() <= 1e-12 * np.abs(Wo).max()
        absent = ~pres
        assert np.all(W[absent] == 0) and np.all(W[:, absent] == 0)


def test_host_patch_matrix_rejects_bad_class():
    with pytest.raises(vk.VkmgError) as e:
        vk.host_patch_matrix(8, 1.0, 0.5, 25)
    assert e.value.status_name == "VKMG_ERR_INVALID_ARG"
    with pytest.raises(vk.VkmgError):
        vk.host_patch_matrix(8, 0.0, 0.5, 12)
