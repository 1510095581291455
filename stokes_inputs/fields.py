"""Problem data for 2D Stokes on the unit square with a uniform N x N quad mesh.

Vector layout used everywhere (the library's ABI layout as well):
``[u_x, u_y, p]``, where ``u_x`` and ``u_y`` hold the values at the
``(2N+1)^2`` biquadratic (Q2) nodes and ``p`` the values at the ``(N+1)^2``
bilinear (Q1) nodes, each block row-major with flat index ``j*side + i``
(``i`` along x).  Q2 node ``(i, j)`` sits at ``(i h/2, j h/2)`` and Q1 node
``(i, j)`` at ``(i h, j h)`` with ``h = 1/N``.

The manufactured solutions satisfy the incompressible Stokes equations
``-nu lap(u) + grad(p) = f``, ``div(u) = 0`` (paper, section "Problem
setup").  ``paper_poly`` is the polynomial solution printed in that section;
``trig`` is the stream-function solution ``u = curl(sin^2(pi x) sin^2(pi y))``,
``p = cos(pi x) cos(pi y)``, which vanishes on the boundary.  Forcing terms
were derived by hand from these definitions; the oracle's convergence-rate
tests are what pin them.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class GridSizes:
    N: int
    q2_side: int
    q1_side: int
    n_q2: int
    n_q1: int
    n_vel: int
    n_pres: int
    n: int
    off_ux: int
    off_uy: int
    off_p: int


def grid_sizes(N: int) -> GridSizes:
    if N < 1:
        raise ValueError("N must be >= 1")
    s2, s1 = 2 * N + 1, N + 1
    n_q2, n_q1 = s2 * s2, s1 * s1
    return GridSizes(N, s2, s1, n_q2, n_q1, 2 * n_q2, n_q1, 2 * n_q2 + n_q1,
                     0, n_q2, 2 * n_q2)


def q2_coords(N: int):
    """(x, y) of every Q2 node, flattened row-major (index j*(2N+1)+i)."""
    t = np.arange(2 * N + 1, dtype=np.float64) / (2.0 * N)
    X, Y = np.meshgrid(t, t, indexing="xy")
    return X.ravel(), Y.ravel()


def q1_coords(N: int):
    t = np.arange(N + 1, dtype=np.float64) / float(N)
    X, Y = np.meshgrid(t, t, indexing="xy")
    return X.ravel(), Y.ravel()


def q2_boundary_mask(N: int) -> np.ndarray:
    s2 = 2 * N + 1
    i = np.arange(s2)
    I, J = np.meshgrid(i, i, indexing="xy")
    return ((I == 0) | (J == 0) | (I == s2 - 1) | (J == s2 - 1)).ravel()


def velocity_dirichlet_mask(N: int) -> np.ndarray:
    """Boolean mask over the full vector: both velocity components at every
    boundary Q2 node (the paper's Dirichlet velocity condition on all edges)."""
    g = grid_sizes(N)
    m = np.zeros(g.n, dtype=bool)
    bm = q2_boundary_mask(N)
    m[g.off_ux:g.off_ux + g.n_q2] = bm
    m[g.off_uy:g.off_uy + g.n_q2] = bm
    return m


# ----------------------------------------------------------------------------
# Manufactured solutions
# ----------------------------------------------------------------------------

def _poly_a(t):
    return t * (1.0 - t) * (2.0 * t - 1.0)


def _poly_c(t):
    return 6.0 * t * t - 6.0 * t + 1.0


class _PaperPoly:
    """u = (a(x) c(y), -a(y) c(x)) with a(t)=t(1-t)(2t-1), c(t)=6t^2-6t+1,
    p = x^2 - 3y^2 + 8xy/3 (zero mean)."""

    name = "paper_poly"

    @staticmethod
    def u(x, y):
        return _poly_a(x) * _poly_c(y), -_poly_a(y) * _poly_c(x)

    @staticmethod
    def grad_u(x, y):
        # d/dt a(t) = -(6t^2-6t+1) = -c(t);  d/dt c(t) = 12t - 6
        ux_x = -_poly_c(x) * _poly_c(y)
        ux_y = _poly_a(x) * (12.0 * y - 6.0)
        uy_x = -_poly_a(y) * (12.0 * x - 6.0)
        uy_y = _poly_c(y) * _poly_c(x)
        return ux_x, ux_y, uy_x, uy_y

    @staticmethod
    def p(x, y):
        return x * x - 3.0 * y * y + (8.0 / 3.0) * x * y

    @staticmethod
    def f(x, y, nu):
        # lap(u_x) = a''(x) c(y) + a(x) c''(y) = (6-12x) c(y) + 12 a(x)
        lap1 = (6.0 - 12.0 * x) * _poly_c(y) + 12.0 * _poly_a(x)
        # lap(u_y) = -[(6-12y) c(x) + 12 a(y)]
        lap2 = -((6.0 - 12.0 * y) * _poly_c(x) + 12.0 * _poly_a(y))
        px = 2.0 * x + (8.0 / 3.0) * y
        py = -6.0 * y + (8.0 / 3.0) * x
        return -nu * lap1 + px, -nu * lap2 + py


class _Trig:
    """psi = sin^2(pi x) sin^2(pi y), u = (d psi/dy, -d psi/dx),
    p = cos(pi x) cos(pi y)."""

    name = "trig"

    @staticmethod
    def u(x, y):
        pi = np.pi
        return (pi * np.sin(pi * x) ** 2 * np.sin(2 * pi * y),
                -pi * np.sin(2 * pi * x) * np.sin(pi * y) ** 2)

    @staticmethod
    def grad_u(x, y):
        pi = np.pi
        ux_x = pi * pi * np.sin(2 * pi * x) * np.sin(2 * pi * y)
        ux_y = 2 * pi * pi * np.sin(pi * x) ** 2 * np.cos(2 * pi * y)
        uy_x = -2 * pi * pi * np.cos(2 * pi * x) * np.sin(pi * y) ** 2
        uy_y = -pi * pi * np.sin(2 * pi * x) * np.sin(2 * pi * y)
        return ux_x, ux_y, uy_x, uy_y

    @staticmethod
    def p(x, y):
        return np.cos(np.pi * x) * np.cos(np.pi * y)

    @staticmethod
    def f(x, y, nu):
        pi = np.pi
        f1 = (-2.0 * nu * pi ** 3 * np.sin(2 * pi * y) * (2 * np.cos(2 * pi * x) - 1)
              - pi * np.sin(pi * x) * np.cos(pi * y))
        f2 = (2.0 * nu * pi ** 3 * np.sin(2 * pi * x) * (2 * np.cos(2 * pi * y) - 1)
              - pi * np.cos(pi * x) * np.sin(pi * y))
        return f1, f2


MANUFACTURED = {"paper_poly": _PaperPoly, "trig": _Trig}


def manufactured_nodal_force(N: int, name: str, nu: float = 1.0) -> np.ndarray:
    """Body force f sampled at the Q2 nodes, shape (2, (2N+1)^2)."""
    X, Y = q2_coords(N)
    f1, f2 = MANUFACTURED[name].f(X, Y, nu)
    return np.stack([f1, f2]).astype(np.float64)


def manufactured_boundary_values(N: int, name: str) -> np.ndarray:
    """Exact velocity at the Q2 nodes, shape (2, (2N+1)^2).  Only the
    boundary entries are used as Dirichlet data."""
    X, Y = q2_coords(N)
    u1, u2 = MANUFACTURED[name].u(X, Y)
    return np.stack([u1, u2]).astype(np.float64)


def manufactured_exact_vector(N: int, name: str) -> np.ndarray:
    """Nodal interpolant of the exact (u, p) in the full vector layout."""
    X2, Y2 = q2_coords(N)
    X1, Y1 = q1_coords(N)
    sol = MANUFACTURED[name]
    u1, u2 = sol.u(X2, Y2)
    return np.concatenate([u1, u2, sol.p(X1, Y1)]).astype(np.float64)


def lid_boundary_values(N: int) -> np.ndarray:
    """Lid-driven cavity data: u = (1, 0) on the top edge at nodes with
    0 < x < 1, zero elsewhere (corners zero so the discrete boundary flux
    vanishes).  Shape (2, (2N+1)^2)."""
    s2 = 2 * N + 1
    g = np.zeros((2, s2, s2))
    g[0, s2 - 1, 1:s2 - 1] = 1.0
    return g.reshape(2, -1)


# ----------------------------------------------------------------------------
# Seeded random data
# ----------------------------------------------------------------------------

def gaussian_random_field(N: int, seed: int, length: float = 0.1,
                          components: int = 2) -> np.ndarray:
    """Smooth Gaussian random field on the Q2 nodal grid.

    White noise N(0,1) from ``numpy.random.default_rng(seed)`` on the
    (2N+1)^2 grid per component, filtered in Fourier space by
    exp(-k^2 length^2 / 2) (k the physical angular wavenumber, grid spacing
    h/2), then rescaled to unit sample variance per component.
    Returns shape (components, (2N+1)^2), float64."""
    s2 = 2 * N + 1
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((components, s2, s2))
    dx = 0.5 / N
    kx = 2.0 * np.pi * np.fft.fftfreq(s2, d=dx)
    ky = 2.0 * np.pi * np.fft.rfftfreq(s2, d=dx)
    K2 = kx[:, None] ** 2 + ky[None, :] ** 2
    filt = np.exp(-0.5 * K2 * length * length)
    out = np.empty_like(w)
    for c in range(components):
        F = np.fft.rfft2(w[c])
        fld = np.fft.irfft2(F * filt, s=(s2, s2))
        fld -= fld.mean()
        fld /= fld.std()
        out[c] = fld
    return out.reshape(components, -1)


def uniform_vector(n: int, seed: int, low: float = -1.0, high: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(low, high, size=n)


def dirichlet_consistent_pair(N: int, seed_x: int = 3, seed_b: int = 4):
    """x, b ~ U[-1,1] with b equal to x on the Dirichlet velocity DoFs, so
    that the residual vanishes there."""
    g = grid_sizes(N)
    x = uniform_vector(g.n, seed_x)
    b = uniform_vector(g.n, seed_b)
    m = velocity_dirichlet_mask(N)
    b[m] = x[m]
    return x, b


def log_viscosity_field(N: int, seed: int) -> np.ndarray:
    """Per-element log-viscosity ~ U[-1,1], shape (N*N,), element index
    ey*N + ex."""
    return uniform_vector(N * N, seed)
