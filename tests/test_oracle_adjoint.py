"""Pin of the oracle's force gradient (chain rule through the symmetric
solve) against central differences of the oracle's own solve.  The loss is
quadratic in f, so central differences are exact up to rounding."""

import numpy as np

from oracle import adjoint
from stokes_inputs import gaussian_random_field, grid_sizes, log_viscosity_field, uniform_vector


def test_force_gradient_matches_central_differences():
    N = 6
    gs = grid_sizes(N)
    f = gaussian_random_field(N, 3, length=0.3)
    xt = uniform_vector(gs.n, 4)

    def loss(ff):
        x = adjoint.solve(N, ff)
        return 0.5 * float(np.sum((x - xt) ** 2))

    x = adjoint.solve(N, f)
    grad = adjoint.force_gradient(N, x - xt)
    rng = np.random.default_rng(8)
    for _ in range(5):
        d = rng.standard_normal(f.shape)
        fd = (loss(f + d) - loss(f - d)) / 2.0
        assert abs(fd - float(np.sum(grad * d))) <= 1e-9 * abs(fd)


def test_pressure_projection_removes_the_null_space_component():
    N = 4
    gs = grid_sizes(N)
    f = gaussian_random_field(N, 5, length=0.3)
    x = adjoint.solve(N, f)
    assert abs(x[gs.off_p:].mean()) < 1e-14
    # the gradient ignores a constant pressure shift in dL/dx
    g = uniform_vector(gs.n, 6)
    g2 = g.copy()
    g2[gs.off_p:] += 3.0
    assert np.allclose(adjoint.force_gradient(N, g), adjoint.force_gradient(N, g2), atol=1e-12)


def test_viscosity_gradient_matches_central_differences():
    """The loss is not quadratic in nu: central differences with a small
    relative step (error O(eps^2))."""
    N = 6
    gs = grid_sizes(N)
    f = gaussian_random_field(N, 3, length=0.3)
    nu = np.exp(log_viscosity_field(N, 7))
    xt = uniform_vector(gs.n, 4)

    def loss(v):
        x = adjoint.solve(N, f, nu=v)
        return 0.5 * float(np.sum((x - xt) ** 2))

    x = adjoint.solve(N, f, nu=nu)
    grad = adjoint.viscosity_gradient(N, x - xt, x, nu)
    rng = np.random.default_rng(8)
    for _ in range(5):
        d = rng.standard_normal(nu.shape) * nu
        eps = 1e-4
        fd = (loss(nu + eps * d) - loss(nu - eps * d)) / (2 * eps)
        assert abs(fd - float(grad @ d)) <= 1e-6 * abs(fd)


def test_iterative_gradients_match_dense_path():
    """The multigrid-FGMRES route to both gradients (for meshes too large for
    dense solves) against the dense bordered solves, per-element viscosity
    log nu ~ U[-1, 1]: solves to rtol 1e-12, gradients within 1e-9."""
    N, levels = 16, 3
    gs = grid_sizes(N)
    f = gaussian_random_field(N, 3, length=0.3)
    nu = np.exp(log_viscosity_field(N, 7))
    xt = uniform_vector(gs.n, 4) * 0.01
    x_hat, gf, gnu, fw, aw = adjoint.iterative_gradients(N, levels, f, lambda x: x - xt, nu,
                                                          rtol=1e-12)
    assert fw.converged and aw.converged
    x = adjoint.solve(N, f, nu=nu)
    assert np.linalg.norm(x_hat - x) <= 1e-9 * np.linalg.norm(x)
    gf_d = adjoint.force_gradient(N, x - xt, nu=nu)
    gnu_d = adjoint.viscosity_gradient(N, x - xt, x, nu)
    assert np.linalg.norm(gf - gf_d) <= 1e-9 * np.linalg.norm(gf_d)
    assert np.linalg.norm(gnu - gnu_d) <= 1e-9 * np.linalg.norm(gnu_d)
