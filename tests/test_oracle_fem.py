"""Pins of the oracle's discretisation against what the mathematics fixes.

Each test checks the oracle by a route other than its own formula:
textbook closed forms, exact reproduction of polynomial solutions, the
divergence of a known field, spectral properties of the saddle-point
matrix and the Taylor-Hood convergence orders.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem
from stokes_inputs import (MANUFACTURED, grid_sizes, manufactured_boundary_values,
                           manufactured_exact_vector, q1_coords, q2_coords,
                           velocity_dirichlet_mask)


def direct_solve(N, A, b, permc="COLAMD"):
    """Exact sparse solve of the consistent singular system with the
    pressure constant fixed by pinning the first pressure DoF to zero."""
    g = grid_sizes(N)
    keep = np.ones(g.n)
    keep[g.off_p] = 0.0
    D = sp.diags(keep)
    Af = (D @ A @ D + sp.diags(1.0 - keep)).tocsc()
    bf = b.copy()
    bf[g.off_p] = 0.0
    return spla.spsolve(Af, bf, permc_spec=permc)


@pytest.mark.parametrize("h", [1.0, 0.25, 1.0 / 7.0])
def test_element_matrices_match_textbook_1d_factors(h):
    # Textbook 1D quadratic Lagrange element on [0,h]: stiffness and mass.
    K1 = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / (3 * h)
    M1 = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) * h / 30
    # Mixed 1D integrals int phi_a psi_b' and int phi_a psi_b (phi linear).
    G = np.array([[-5 / 6, 2 / 3, 1 / 6], [-1 / 6, -2 / 3, 5 / 6]])
    Mq = np.array([[1, 2, 0], [0, 2, 1]]) * h / 6
    E = fem.element_matrices(h)
    # local index b*3+a (a along x) -> kron(y-factor, x-factor)
    assert np.allclose(E["L"], np.kron(M1, K1) + np.kron(K1, M1), rtol=0, atol=1e-14)
    assert np.allclose(E["M"], np.kron(M1, M1), rtol=0, atol=1e-15)
    assert np.allclose(E["Bx"], -np.kron(Mq, G), rtol=0, atol=1e-14)
    assert np.allclose(E["By"], -np.kron(G, Mq), rtol=0, atol=1e-14)
    # constants are in the kernel of the element Laplacian
    assert np.abs(E["L"].sum(axis=1)).max() < 1e-13
    assert np.allclose(E["wp"], np.full(4, h * h / 4))


@pytest.mark.parametrize("N", [2, 4])
def test_assembled_matrix_symmetry_nullspace_inertia(N):
    g = grid_sizes(N)
    A, _, dmask, _ = fem.stokes_system(N, 1.0)
    assert abs(A - A.T).max() == 0.0
    z = np.zeros(g.n)
    z[g.off_p:] = 1.0
    assert np.abs(A @ z).max() < 1e-13
    ev = np.linalg.eigvalsh(A.toarray())
    tol = 1e-10 * np.abs(ev).max()
    npos, nneg, nzero = (ev > tol).sum(), (ev < -tol).sum(), (np.abs(ev) <= tol).sum()
    # symmetric indefinite saddle point: velocity block SPD (identity rows on
    # the Dirichlet set included), n_p - 1 negative, one constant-pressure
    # null vector
    assert (npos, nneg, nzero) == (g.n_vel, g.n_pres - 1, 1)


@pytest.mark.parametrize("N", [3, 8])
def test_divergence_block_sign_and_scale(N):
    # Before boundary conditions, B applied to the interpolant of u = (x, 0)
    # (div u = 1) gives -int phi_k, which is h^2 times 1, 1/2, 1/4 for
    # interior, edge and corner Q1 nodes.
    g = grid_sizes(N)
    A = fem.assemble_stokes(N, 1.0)
    X, _ = q2_coords(N)
    u = np.zeros(g.n)
    u[g.off_ux:g.off_ux + g.n_q2] = X
    div = (A @ u)[g.off_p:]
    h = 1.0 / N
    I1 = np.arange(N + 1)
    wx = np.where((I1 == 0) | (I1 == N), 0.5, 1.0)
    expect = -h * h * np.outer(wx, wx).ravel()
    assert np.allclose(div, expect, rtol=0, atol=1e-15)


def _solve_polynomial_case(N, u_fn, p_fn, f_fn, nu=1.0):
    g = grid_sizes(N)
    X2, Y2 = q2_coords(N)
    X1, Y1 = q1_coords(N)
    b_load = fem.rhs_from_function(N, lambda x, y, nu_: f_fn(x, y), nu)
    u1, u2 = u_fn(X2, Y2)
    gnod = np.stack([u1, u2])
    A, b, dmask, _ = fem.stokes_system(N, nu, b_load=b_load, g_nodal=gnod)
    x = direct_solve(N, A, b)
    x = fem.normalise_pressure(N, x)
    exact = np.concatenate([u1, u2, p_fn(X1, Y1)])
    exact = fem.normalise_pressure(N, exact)
    return x, exact


@pytest.mark.parametrize("N", [2, 5])
def test_exact_for_solutions_in_the_discrete_space(N):
    # u = (y^2, 0), p = 0 satisfies div u = 0 and -lap u = (-2, 0); it lies
    # in Q2 x Q1, so the discrete solution is its interpolant.
    x, ex = _solve_polynomial_case(
        N, lambda X, Y: (Y * Y, 0 * X), lambda X, Y: 0 * X,
        lambda X, Y: (-2.0 + 0 * X, 0 * X))
    assert np.abs(x - ex).max() < 1e-10  # rounding of a solve with cond ~ 1e4
    # u = 0, p = (x-1/2)(y-1/2): f = grad p.
    x, ex = _solve_polynomial_case(
        N, lambda X, Y: (0 * X, 0 * X), lambda X, Y: (X - 0.5) * (Y - 0.5),
        lambda X, Y: (Y - 0.5, X - 0.5))
    assert np.abs(x - ex).max() < 1e-10  # rounding of a solve with cond ~ 1e4


@pytest.mark.parametrize("name", ["paper_poly", "trig"])
@pytest.mark.parametrize("rhs", ["quadrature", "nodal"])
def test_taylor_hood_convergence_orders(name, rhs):
    errs = []
    Ns = [8, 16, 32, 64]
    for N in Ns:
        if rhs == "quadrature":
            b_load = fem.rhs_from_function(N, MANUFACTURED[name].f, 1.0)
            A, b, _, _ = fem.stokes_system(N, 1.0, b_load=b_load,
                                           g_nodal=manufactured_boundary_values(N, name))
        else:
            from stokes_inputs import manufactured_nodal_force
            A, b, _, _ = fem.stokes_system(N, 1.0, f_nodal=manufactured_nodal_force(N, name),
                                           g_nodal=manufactured_boundary_values(N, name))
        x = direct_solve(N, A, b)
        errs.append(fem.discretisation_errors(N, x, name))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    # velocity L2 -> 3, velocity H1 -> 2, pressure L2 -> 2 (at least)
    assert rates[-1, 0] > 2.8, rates
    assert rates[-1, 1] > 1.9, rates
    assert rates[-1, 2] > 1.8, rates


def test_dirichlet_elimination_is_symmetric_and_lifts():
    N = 4
    g = grid_sizes(N)
    gnod = manufactured_boundary_values(N, "paper_poly")
    A_full = fem.assemble_stokes(N)
    A, b, dmask, xl = fem.stokes_system(N, 1.0, g_nodal=gnod)
    assert abs(A - A.T).max() == 0.0
    assert np.array_equal(dmask, velocity_dirichlet_mask(N))
    # rows of D are identity, b_D = g
    Ad = A.toarray()
    assert np.array_equal(Ad[dmask][:, dmask], np.eye(dmask.sum()))
    assert np.all(Ad[dmask][:, ~dmask] == 0)
    assert np.allclose(b[dmask], xl[dmask])
    # with zero load, for any x with x_D = g the constrained residual on the
    # free rows equals the unconstrained operator's free rows
    rng = np.random.default_rng(0)
    x = rng.standard_normal(g.n)
    x[dmask] = xl[dmask]
    lhs = (A @ x - b)[~dmask]
    rhs = (A_full @ x)[~dmask]  # load is zero here
    assert np.allclose(lhs, rhs, atol=1e-13)
