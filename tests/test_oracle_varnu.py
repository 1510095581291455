"""Pins of the oracle's per-element viscosity path (the variable-coefficient
extension for which the shared-inverse Vanka does not apply): assembly,
coarse-level averaging, per-patch ("simple") Vanka and multigrid."""

import numpy as np

from oracle import fem, fgmres, multigrid, vanka
from stokes_inputs import grid_sizes, log_viscosity_field, velocity_dirichlet_mask


def _nu(N, seed=7):
    return np.exp(log_viscosity_field(N, seed))


def test_variable_viscosity_assembly():
    N = 6
    g = grid_sizes(N)
    nu = _nu(N)
    A = fem.assemble_stokes(N, nu).toarray()
    assert np.allclose(A, A.T)
    L = A[:g.off_uy, :g.off_uy]
    # constants lie in the kernel of every element Laplacian
    assert np.abs(L @ np.ones(g.n_q2)).max() < 1e-12 * np.abs(L).max()
    # a constant field equals the scalar assembly; linear in nu
    assert np.allclose(fem.assemble_stokes(N, np.full(N * N, 2.5)).toarray(),
                       fem.assemble_stokes(N, 2.5).toarray())
    A2 = fem.assemble_stokes(N, 2.0 * nu).toarray()
    assert np.allclose(A2[:g.off_p, :g.off_p], 2.0 * A[:g.off_p, :g.off_p])
    assert np.allclose(A2[g.off_p:, :], A[g.off_p:, :])
    # energy: u^T L u = sum_e nu_e u_e^T L_e u_e >= 0 and zero only for constants
    rng = np.random.default_rng(1)
    u = rng.standard_normal(g.n_q2)
    assert u @ L @ u > 0


def test_coarse_viscosity_is_the_mean_of_the_children():
    N, levels = 16, 3
    nu = _nu(N)
    H = multigrid.Hierarchy(N, levels, nu=nu)
    for l in range(levels):
        Nl = N >> (levels - 1 - l)
        assert np.size(H.nu_levels[l]) == Nl * Nl
        assert np.isclose(np.mean(H.nu_levels[l]), np.mean(nu))
    f = np.asarray(H.nu_levels[2]).reshape(16, 16)
    c = np.asarray(H.nu_levels[1]).reshape(8, 8)
    assert np.isclose(c[3, 5], f[6:8, 10:12].mean())


def test_simple_vanka_patches_invert_their_own_blocks():
    N = 8
    nu = _nu(N)
    A, _, dm, _ = fem.stokes_system(N, nu)
    sm = vanka.VankaSmoother(A, N, dm, 0.5, shared=False)
    idx = vanka.patch_dofs(N)
    for k in (0, 5, 30, 40, 60, 80):
        dofs = idx[k]
        pres = dofs >= 0
        Ai = vanka.extract_patch_matrix(A, dofs)
        Bi = sm.inv[k][np.ix_(pres, pres)]
        assert np.allclose(Ai @ Bi, np.eye(int(pres.sum())), atol=1e-10)
    # variable viscosity makes interior patches differ
    assert not np.allclose(sm.inv[40], sm.inv[41])


def test_variable_viscosity_multigrid_contracts_and_solves():
    N, levels = 16, 3
    nu = _nu(N)
    H = multigrid.Hierarchy(N, levels, nu=nu)
    A = H.A
    n = A.shape[0]
    off_p = grid_sizes(N).off_p
    dm = velocity_dirichlet_mask(N)
    rng = np.random.default_rng(3)
    e = rng.standard_normal(n)
    e[dm] = 0.0
    for _ in range(10):
        e2 = e - H.vcycle(A @ e)
        e2[off_p:] -= e2[off_p:].mean()
        rho = np.linalg.norm(e2) / np.linalg.norm(e)
        e = e2 / np.linalg.norm(e2)
    assert rho < 0.6
    xt = rng.standard_normal(n)
    xt[dm] = 0.0
    xt[off_p:] -= xt[off_p:].mean()
    res = fgmres.fgmres(A, A @ xt, np.zeros(n), H.vcycle, rtol=1e-10, restart=30, max_iters=80)
    assert res.converged
    xs = res.x.copy()
    xs[off_p:] -= xs[off_p:].mean()
    # the viscosity contrast (e^2) worsens the conditioning: error ~ cond * rtol
    assert np.linalg.norm(xs - xt) <= 1e-7 * np.linalg.norm(xt)


def test_galerkin_coarse_operator_equals_rediscretisation_for_constant_viscosity():
    """Nested Q2-Q1 spaces: with a constant viscosity the product P^T A P is
    the coarse finite-element operator itself, so both hierarchies hold the
    same matrices and give the same V-cycle."""
    N, levels = 16, 3
    Hr = multigrid.Hierarchy(N, levels)
    Hg = multigrid.Hierarchy(N, levels, coarse_operator="galerkin")
    for lr, lg in zip(Hr.levels, Hg.levels):
        d = abs(lr.A - lg.A).max()
        assert d <= 1e-12 * abs(lr.A).max()
    r = np.random.default_rng(4).standard_normal(Hr.A.shape[0])
    r[velocity_dirichlet_mask(N)] = 0.0
    zr, zg = Hr.vcycle(r), Hg.vcycle(r)
    assert np.abs(zr - zg).max() <= 1e-10 * np.abs(zr).max()


def test_galerkin_coarse_operator_of_blockwise_viscosity_is_the_coarse_assembly():
    """A viscosity that is constant on each 2x2 block of fine elements is a
    coarse-element field; the coarse integrals are then exactly the sums of
    the fine ones, so P^T A P equals the coarse finite-element assembly with
    that field (an identity of the discretisation, independent of P's
    construction)."""
    N, levels = 8, 2
    nc = _nu(N // 2, seed=9).reshape(N // 2, N // 2)
    nf = np.repeat(np.repeat(nc, 2, axis=0), 2, axis=1).ravel()
    Hg = multigrid.Hierarchy(N, levels, nu=nf, coarse_operator="galerkin")
    Ac, _, _, _ = fem.stokes_system(N // 2, nc.ravel())
    d = abs(Hg.levels[0].A - Ac).max()
    assert d <= 1e-12 * abs(Ac).max()


def test_galerkin_coarse_operator_structure_for_variable_viscosity():
    """Symmetric, constant-pressure null space, identity Dirichlet rows, and
    couplings only between DoFs of a common coarse element (the pattern of
    a coarse assembly with a generic per-element viscosity, which has no
    exact cancellations), so the Vanka patches see the same local
    structure."""
    N, levels = 16, 3
    Hg = multigrid.Hierarchy(N, levels, nu=_nu(N), coarse_operator="galerkin")
    for l in range(levels - 1):
        Nl = Hg.levels[l].N
        A = Hg.levels[l].A
        g = grid_sizes(Nl)
        assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
        c = np.zeros(g.n)
        c[g.off_p:] = 1.0
        assert np.abs(A @ c).max() <= 1e-12 * abs(A).max()
        dm = velocity_dirichlet_mask(Nl)
        Ad = A.toarray()
        assert np.array_equal(Ad[dm][:, dm], np.eye(int(dm.sum())))
        assert not np.any(Ad[dm][:, ~dm]) and not np.any(Ad[~dm][:, dm])
        Ar, _, _, _ = fem.stokes_system(Nl, _nu(Nl, seed=11))
        # entries outside it are rounding residue of exact cancellations
        outside = np.abs(Ad[Ar.toarray() == 0])
        assert outside.max(initial=0.0) <= 1e-14 * np.abs(Ad).max()
