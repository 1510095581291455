"""Thin ctypes binding of the vkmg C ABI (include/vkmg.h).

Argument marshalling only: every numerical step runs in the HIP library
``libvkmg.so`` built in this directory.  PyTorch supplies device memory
(``tensor.data_ptr()``) and the current HIP stream.  There is no fallback:
if the library is missing, loading raises.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int32, c_int64, c_uint8, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvkmg.so")

FP64, FP32 = 0, 1
APPLY = {"vector": 0, "matrix": 1}
RELAX = {"vanka": 0, "braess_sarazin": 1}
(KERNEL_VANKA, KERNEL_RESIDUAL, KERNEL_TRANSFER, KERNEL_COARSE, KERNEL_KRYLOV,
 KERNEL_VANKA_TILE) = range(6)

STATUS = {
    0: "VKMG_OK",
    1: "VKMG_ERR_INVALID_ARG",
    2: "VKMG_ERR_UNSUPPORTED",
    3: "VKMG_ERR_OUT_OF_MEMORY",
    4: "VKMG_ERR_HIP",
    5: "VKMG_ERR_SINGULAR_PATCH",
    6: "VKMG_ERR_NOT_CONVERGED",
    7: "VKMG_ERR_NONFINITE",
}

EXPORTED = [
    "vkmg_default_options", "vkmg_setup", "vkmg_setup_viscosity", "vkmg_destroy", "vkmg_layout_of", "vkmg_level_layout",
    "vkmg_num_levels", "vkmg_residual", "vkmg_apply", "vkmg_assemble_rhs", "vkmg_vanka_sweep",
    "vkmg_vanka_update", "vkmg_vanka_update_noalloc", "vkmg_relax", "vkmg_assemble_rhs_adjoint", "vkmg_remove_pressure_mean", "vkmg_dirichlet_lift",
    "vkmg_viscosity_gradient",
    "vkmg_restrict", "vkmg_prolong_add", "vkmg_coarse_solve", "vkmg_vcycle",
    "vkmg_fgmres_solve", "vkmg_get_tuning", "vkmg_set_tuning", "vkmg_autotune", "vkmg_set_timing", "vkmg_kernel_timing", "vkmg_host_patch_matrix",
    "vkmg_status_string", "vkmg_last_error",
]


class VkmgError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.status_name}: {message}")


class Grid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("nu_pre", c_int32), ("nu_post", c_int32), ("omega", c_double),
                ("mg_precision", c_int32), ("interior_apply", c_int32), ("use_graphs", c_int32),
                ("batch", c_int32), ("relaxation", c_int32), ("bs_t", c_double),
                ("bs_omega", c_double), ("bs_jacobi_weight", c_double),
                ("bs_jacobi_sweeps", c_int32)]


class Layout(ctypes.Structure):
    _fields_ = [("n", c_int64), ("n_vel", c_int64), ("n_pres", c_int64), ("off_ux", c_int64),
                ("off_uy", c_int64), ("off_p", c_int64), ("q2_side", c_int32),
                ("q1_side", c_int32), ("n_elem", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("fused_sweep_max_n", c_int32), ("park_min_n", c_int32),
                ("fused_prolong_max_n", c_int32), ("boundary_per_wave", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("restarts", c_int32), ("est_rel_res", c_double),
                ("true_rel_res", c_double), ("status", c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libvkmg.so and declare its signatures (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run: python -m paper_2401_06277_amd.build)")
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "vkmg_default_options": (Options, []),
        "vkmg_setup": (c_int32, [POINTER(Grid), c_int32, c_double, POINTER(Options), P, POINTER(P)]),
        "vkmg_setup_viscosity": (c_int32, [POINTER(Grid), c_int32, P, POINTER(Options), P, POINTER(P)]),
        "vkmg_destroy": (None, [P]),
        "vkmg_layout_of": (c_int32, [P, POINTER(Layout)]),
        "vkmg_level_layout": (c_int32, [P, c_int32, POINTER(Layout)]),
        "vkmg_num_levels": (c_int32, [P, POINTER(c_int32)]),
        "vkmg_residual": (c_int32, [P, P, P, P, P]),
        "vkmg_apply": (c_int32, [P, P, P, P]),
        "vkmg_assemble_rhs": (c_int32, [P, P, P, P, P]),
        "vkmg_vanka_sweep": (c_int32, [P, c_int32, P, P, P]),
        "vkmg_vanka_update": (c_int32, [P, c_int32, P, P, P]),
        "vkmg_vanka_update_noalloc": (c_int32, [P, c_int32, P, P, P]),
        "vkmg_relax": (c_int32, [P, c_int32, P, P, P]),
        "vkmg_assemble_rhs_adjoint": (c_int32, [P, P, P, P]),
        "vkmg_remove_pressure_mean": (c_int32, [P, P, P]),
        "vkmg_dirichlet_lift": (c_int32, [P, P, P, P]),
        "vkmg_viscosity_gradient": (c_int32, [P, P, P, P, P]),
        "vkmg_restrict": (c_int32, [P, c_int32, P, P, P]),
        "vkmg_prolong_add": (c_int32, [P, c_int32, P, P, P]),
        "vkmg_coarse_solve": (c_int32, [P, P, P, P]),
        "vkmg_vcycle": (c_int32, [P, P, P, P]),
        "vkmg_fgmres_solve": (c_int32, [P, P, P, c_double, c_int32, c_int32, POINTER(Info), P]),
        "vkmg_get_tuning": (c_int32, [P, POINTER(Tuning)]),
        "vkmg_set_tuning": (c_int32, [P, POINTER(Tuning)]),
        "vkmg_autotune": (c_int32, [P, c_int32, P, POINTER(Tuning)]),
        "vkmg_set_timing": (c_int32, [P, c_int32]),
        "vkmg_kernel_timing": (c_int32, [P, c_int32, c_int32, POINTER(c_int64), POINTER(c_double)]),
        "vkmg_host_patch_matrix": (c_int32, [c_int32, c_double, c_double, c_int32, P, P, P, P]),
        "vkmg_status_string": (c_char_p, [c_int32]),
        "vkmg_last_error": (c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        msg = _lib.vkmg_last_error().decode(errors="replace")
        raise VkmgError(status, where, msg)


def host_patch_matrix(N: int, nu: float, omega: float, cls: int):
    """Patch matrix, inverse and weighted inverse of patch class ``cls`` (host
    only, no GPU).  Returns (A, Ainv, Wainv, present) as numpy arrays."""
    lib = load_library()
    A = np.zeros((51, 51))
    Ai = np.zeros((51, 51))
    W = np.zeros((51, 51))
    pres = np.zeros(51, dtype=np.uint8)
    st = lib.vkmg_host_patch_matrix(N, nu, omega, cls, A.ctypes.data, Ai.ctypes.data,
                                    W.ctypes.data, pres.ctypes.data)
    _check(st, "vkmg_host_patch_matrix")
    return A, Ai, W, pres.astype(bool)


def default_options():
    return load_library().vkmg_default_options()


class VkmgSolver:
    """One vkmg context: the multigrid hierarchy of an N x N Q2-Q1 Stokes
    problem on the current HIP device.  With ``batch`` > 1 every vector
    argument holds ``batch`` vectors back to back (a tensor of batch * size
    elements, e.g. shape (batch, size)) and fgmres_solve returns a list of
    info dicts."""

    def __init__(self, N: int, levels: int, nu: float = 1.0, nu_pre: int = 2, nu_post: int = 2,
                 omega: float = 0.5, precision: str = "fp64", interior_apply: str = "vector",
                 graphs: bool = True, batch: int = 1, relaxation: str = "vanka",
                 bs_t: float = 1.0, bs_omega: float = 1.0, bs_jacobi_weight: float = 1.0,
                 bs_jacobi_sweeps: int = 2, nu_elem=None):
        import torch
        lib = load_library()
        self._torch = torch
        self.precision = precision
        self.interior_apply = interior_apply
        if interior_apply not in APPLY:
            raise ValueError(f"interior_apply must be one of {sorted(APPLY)}")
        if relaxation not in RELAX:
            raise ValueError(f"relaxation must be one of {sorted(RELAX)}")
        opts = Options(nu_pre, nu_post, omega, FP32 if precision == "fp32" else FP64,
                       APPLY[interior_apply], 1 if graphs else 0, batch, RELAX[relaxation],
                       bs_t, bs_omega, bs_jacobi_weight, bs_jacobi_sweeps)
        ctx = c_void_p()
        if nu_elem is None:
            st = lib.vkmg_setup(byref(Grid(N, N)), levels, nu, byref(opts), self._stream(),
                                byref(ctx))
            _check(st, "vkmg_setup")
        else:
            # per-element viscosity (host array of N*N values, index ey*N + ex)
            arr = np.ascontiguousarray(np.asarray(nu_elem, dtype=np.float64).ravel())
            if arr.size != N * N:
                raise ValueError(f"nu_elem must have {N * N} values")
            st = lib.vkmg_setup_viscosity(byref(Grid(N, N)), levels,
                                          arr.ctypes.data_as(c_void_p), byref(opts),
                                          self._stream(), byref(ctx))
            _check(st, "vkmg_setup_viscosity")
        self.nu_elem = None if nu_elem is None else arr
        self._ctx = ctx
        self.N, self.levels, self.nu, self.batch = N, levels, nu, batch
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.mg_dtype = torch.float32 if precision == "fp32" else torch.float64
        # the field on the device, for the identity check of the tensors
        # passed to the differentiable solve (check_viscosity)
        self._nu_dev = None if nu_elem is None else torch.from_numpy(arr).to(self.device)
        self._nu_checked = None

    # ---------------------------------------------------------------- plumbing
    def _stream(self):
        import torch
        return c_void_p(torch.cuda.current_stream().cuda_stream)

    def _ptr(self, t, dtype, n=None, name="tensor"):
        if not t.is_cuda or t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if n is not None and t.numel() != n:
            raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
        return c_void_p(t.data_ptr())

    def _empty(self, n, dtype):
        return self._torch.empty(n, dtype=dtype, device=self.device)

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _lib.vkmg_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def check_viscosity(self, nu):
        """Raise unless `nu` (a device tensor of N*N values) holds the
        per-element viscosity this context was set up with.  Compared on the
        device, once per tensor version (no host copy)."""
        if self._nu_dev is None:
            raise ValueError("nu given but the solver has a constant viscosity")
        key = (nu.data_ptr(), nu._version, nu.numel(), str(nu.device))
        if key == self._nu_checked:
            return
        if nu.numel() != self._nu_dev.numel() or not self._torch.equal(
                nu.detach().reshape(-1).to(self._nu_dev.device, self._torch.float64), self._nu_dev):
            raise ValueError("nu differs from the field the solver was set up with")
        self._nu_checked = key

    # ---------------------------------------------------------------- queries
    @property
    def layout(self):
        lay = Layout()
        _check(_lib.vkmg_layout_of(self._ctx, byref(lay)), "vkmg_layout_of")
        return lay.as_dict()

    def level_layout(self, level: int):
        lay = Layout()
        _check(_lib.vkmg_level_layout(self._ctx, level, byref(lay)), "vkmg_level_layout")
        return lay.as_dict()

    @property
    def num_levels(self):
        v = c_int32()
        _check(_lib.vkmg_num_levels(self._ctx, byref(v)), "vkmg_num_levels")
        return v.value

    # ---------------------------------------------------------------- operations
    def residual(self, b, x, r=None):
        n = self.layout["n"] * self.batch
        r = self._empty(n, self._torch.float64) if r is None else r
        st = _lib.vkmg_residual(self._ctx, self._ptr(b, self._torch.float64, n, "b"),
                                self._ptr(x, self._torch.float64, n, "x"),
                                self._ptr(r, self._torch.float64, n, "r"), self._stream())
        _check(st, "vkmg_residual")
        return r

    def apply(self, x, y=None):
        n = self.layout["n"] * self.batch
        y = self._empty(n, self._torch.float64) if y is None else y
        st = _lib.vkmg_apply(self._ctx, self._ptr(x, self._torch.float64, n, "x"),
                             self._ptr(y, self._torch.float64, n, "y"), self._stream())
        _check(st, "vkmg_apply")
        return y

    def assemble_rhs(self, f, g=None, b=None):
        lay = self.layout
        nb = self.batch
        b = self._empty(lay["n"] * nb, self._torch.float64) if b is None else b
        gp = (c_void_p(None) if g is None
              else self._ptr(g, self._torch.float64, lay["n_vel"] * nb, "g"))
        st = _lib.vkmg_assemble_rhs(self._ctx,
                                    self._ptr(f, self._torch.float64, lay["n_vel"] * nb, "f"),
                                    gp, self._ptr(b, self._torch.float64, lay["n"] * nb, "b"),
                                    self._stream())
        _check(st, "vkmg_assemble_rhs")
        return b

    def dirichlet_lift(self, b, x=None):
        """x = b on the Dirichlet DoFs, 0 elsewhere (vkmg_dirichlet_lift):
        the initial guess vkmg_fgmres_solve expects for right-hand side b."""
        n = self.layout["n"] * self.batch
        x = self._empty(n, self._torch.float64) if x is None else x
        st = _lib.vkmg_dirichlet_lift(self._ctx, self._ptr(b, self._torch.float64, n, "b"),
                                      self._ptr(x, self._torch.float64, n, "x"), self._stream())
        _check(st, "vkmg_dirichlet_lift")
        return x

    def assemble_rhs_adjoint(self, lam, grad_f=None):
        """Transpose of the force-to-load map of assemble_rhs applied to lam."""
        lay = self.layout
        nb = self.batch
        grad_f = self._empty(lay["n_vel"] * nb, self._torch.float64) if grad_f is None else grad_f
        st = _lib.vkmg_assemble_rhs_adjoint(
            self._ctx, self._ptr(lam, self._torch.float64, lay["n"] * nb, "lam"),
            self._ptr(grad_f, self._torch.float64, lay["n_vel"] * nb, "grad_f"), self._stream())
        _check(st, "vkmg_assemble_rhs_adjoint")
        return grad_f

    def viscosity_gradient(self, lam, x, grad_nu=None):
        """-lam_e^T L_e x_e per element (N*N values per right-hand side)."""
        n = self.layout["n"] * self.batch
        ne = self.N * self.N * self.batch
        grad_nu = self._empty(ne, self._torch.float64) if grad_nu is None else grad_nu
        st = _lib.vkmg_viscosity_gradient(
            self._ctx, self._ptr(lam, self._torch.float64, n, "lam"),
            self._ptr(x, self._torch.float64, n, "x"),
            self._ptr(grad_nu, self._torch.float64, ne, "grad_nu"), self._stream())
        _check(st, "vkmg_viscosity_gradient")
        return grad_nu

    def remove_pressure_mean(self, x):
        """In place: subtract the mean of the pressure block (per right-hand side)."""
        st = _lib.vkmg_remove_pressure_mean(
            self._ctx, self._ptr(x, self._torch.float64, self.layout["n"] * self.batch, "x"),
            self._stream())
        _check(st, "vkmg_remove_pressure_mean")
        return x

    def vanka_sweep(self, level: int, x, b):
        n = self.level_layout(level)["n"] * self.batch
        st = _lib.vkmg_vanka_sweep(self._ctx, level, self._ptr(x, self.mg_dtype, n, "x"),
                                   self._ptr(b, self.mg_dtype, n, "b"), self._stream())
        _check(st, "vkmg_vanka_sweep")
        return x

    def vanka_update(self, level: int, x, r):
        """x += sum_i V_i^T W_i A_i^{-1} V_i r (the update half of a sweep)."""
        n = self.level_layout(level)["n"] * self.batch
        st = _lib.vkmg_vanka_update(self._ctx, level, self._ptr(x, self.mg_dtype, n, "x"),
                                    self._ptr(r, self.mg_dtype, n, "r"), self._stream())
        _check(st, "vkmg_vanka_update")
        return x

    def vanka_update_noalloc(self, level: int, x, r):
        """vanka_update through the allocation-free entry point (patch
        corrections in the library's static device scratch)."""
        n = self.level_layout(level)["n"] * self.batch
        st = _lib.vkmg_vanka_update_noalloc(self._ctx, level, self._ptr(x, self.mg_dtype, n, "x"),
                                            self._ptr(r, self.mg_dtype, n, "r"), self._stream())
        _check(st, "vkmg_vanka_update_noalloc")
        return x

    def relax(self, level: int, x, b):
        """One sweep of the configured relaxation (Vanka or Braess-Sarazin)."""
        n = self.level_layout(level)["n"] * self.batch
        st = _lib.vkmg_relax(self._ctx, level, self._ptr(x, self.mg_dtype, n, "x"),
                             self._ptr(b, self.mg_dtype, n, "b"), self._stream())
        _check(st, "vkmg_relax")
        return x

    def restrict(self, level: int, r_fine, b_coarse=None):
        nf = self.level_layout(level)["n"] * self.batch
        nc = self.level_layout(level - 1)["n"] * self.batch
        b_coarse = self._empty(nc, self.mg_dtype) if b_coarse is None else b_coarse
        st = _lib.vkmg_restrict(self._ctx, level, self._ptr(r_fine, self.mg_dtype, nf, "r_fine"),
                                self._ptr(b_coarse, self.mg_dtype, nc, "b_coarse"), self._stream())
        _check(st, "vkmg_restrict")
        return b_coarse

    def prolong_add(self, level: int, e_coarse, x_fine):
        nf = self.level_layout(level)["n"] * self.batch
        nc = self.level_layout(level - 1)["n"] * self.batch
        st = _lib.vkmg_prolong_add(self._ctx, level, self._ptr(e_coarse, self.mg_dtype, nc, "e_coarse"),
                                   self._ptr(x_fine, self.mg_dtype, nf, "x_fine"), self._stream())
        _check(st, "vkmg_prolong_add")
        return x_fine

    def coarse_solve(self, r, e=None):
        n0 = self.level_layout(0)["n"] * self.batch
        e = self._empty(n0, self.mg_dtype) if e is None else e
        st = _lib.vkmg_coarse_solve(self._ctx, self._ptr(r, self.mg_dtype, n0, "r"),
                                    self._ptr(e, self.mg_dtype, n0, "e"), self._stream())
        _check(st, "vkmg_coarse_solve")
        return e

    def vcycle(self, r, z=None):
        n = self.layout["n"] * self.batch
        z = self._empty(n, self._torch.float64) if z is None else z
        st = _lib.vkmg_vcycle(self._ctx, self._ptr(r, self._torch.float64, n, "r"),
                              self._ptr(z, self._torch.float64, n, "z"), self._stream())
        _check(st, "vkmg_vcycle")
        return z

    def fgmres_solve(self, b, x, rtol: float = 1e-8, restart: int = 30, max_iters: int = 500,
                     raise_on_error: bool = False):
        """Solve in place (x: initial guess in, solution out).  Returns the
        info dict; NOT_CONVERGED and NONFINITE are reported in it (and raised
        when ``raise_on_error``).  Batched contexts: a list of ``batch``
        info dicts, one per right-hand side."""
        n = self.layout["n"] * self.batch
        info = (Info * self.batch)()
        st = _lib.vkmg_fgmres_solve(self._ctx, self._ptr(b, self._torch.float64, n, "b"),
                                    self._ptr(x, self._torch.float64, n, "x"), rtol, restart,
                                    max_iters, info, self._stream())
        if st not in (0, 6, 7) or (raise_on_error and st != 0):
            _check(st, "vkmg_fgmres_solve")
        if self.batch == 1:
            return info[0].as_dict()
        return [i.as_dict() for i in info]

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(_lib.vkmg_get_tuning(self._ctx, byref(t)), "vkmg_get_tuning")
        return t.as_dict()

    def set_tuning(self, **fields) -> dict:
        """Change launch shapes (vkmg_tuning fields by name); returns the new tuning."""
        t = Tuning(**{**self.get_tuning(), **fields})
        _check(_lib.vkmg_set_tuning(self._ctx, byref(t)), "vkmg_set_tuning")
        return self.get_tuning()

    def autotune(self, reps: int = 10) -> dict:
        """Measure the launch shapes on this GPU (vkmg_autotune); returns them."""
        t = Tuning()
        _check(_lib.vkmg_autotune(self._ctx, reps, self._stream(), byref(t)), "vkmg_autotune")
        return t.as_dict()

    def set_timing(self, class_mask: int):
        _check(_lib.vkmg_set_timing(self._ctx, class_mask), "vkmg_set_timing")

    def kernel_timing(self, kernel_class: int, level: int = -1):
        """(launches, total milliseconds) recorded for a kernel class on one
        level (-1: all levels) since the last set_timing."""
        n = c_int64()
        ms = c_double()
        _check(_lib.vkmg_kernel_timing(self._ctx, kernel_class, level, byref(n), byref(ms)),
               "vkmg_kernel_timing")
        return n.value, ms.value
