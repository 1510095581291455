"""Pins of the oracle's transfers, Vanka patches, V-cycle and FGMRES.

Sources of truth: exact reproduction of coarse polynomials by the
interpolation, the Galerkin identity for nested conforming spaces, the
paper's count of 25 distinct patch matrices on a uniform mesh and its
Table 1 patch sizes (tests/golden/table1_vanka_counts.txt), exact patch
inverses, the multiplicity structure of the overlap, agreement of the
shared-inverse ("tuned") and per-patch ("simple") forms, dense direct
solves, and the minimisation property of GMRES checked by brute-force
least squares.
"""

import os

import numpy as np
import pytest

from oracle import fem, fgmres, multigrid, transfer, vanka
from stokes_inputs import (grid_sizes, manufactured_boundary_values, manufactured_nodal_force,
                           q1_coords, q2_coords, velocity_dirichlet_mask)

from test_oracle_fem import direct_solve


# ---------------------------------------------------------------- transfers

@pytest.mark.parametrize("nc", [1, 2, 5])
def test_prolongation_reproduces_coarse_polynomials(nc):
    gc, gf = grid_sizes(nc), grid_sizes(2 * nc)
    P = transfer.prolongation(nc)
    # biquadratic vanishing on the boundary lies in the coarse Q2 space
    def uq(X, Y):
        return X * (1 - X) * Y * (1 - Y) * (1 + 0 * X)

    def pl(X, Y):
        return 1.0 + 2.0 * X - 3.0 * Y + 4.0 * X * Y

    Xc, Yc = q2_coords(nc)
    Xf, Yf = q2_coords(2 * nc)
    X1c, Y1c = q1_coords(nc)
    X1f, Y1f = q1_coords(2 * nc)
    xc = np.concatenate([uq(Xc, Yc), 2 * uq(Xc, Yc), pl(X1c, Y1c)])
    xf = P @ xc
    expect = np.concatenate([uq(Xf, Yf), 2 * uq(Xf, Yf), pl(X1f, Y1f)])
    assert np.abs(xf - expect).max() < 1e-15 * 8
    # pressure rows sum to one (partition of unity)
    Pp = P[gf.off_p:, gc.off_p:]
    assert np.allclose(np.asarray(Pp.sum(axis=1)).ravel(), 1.0, atol=1e-15)


def test_1d_interpolation_weights():
    # a fine node at 1/4 of a coarse element takes (3/8, 3/4, -1/8) from the
    # coarse (left, mid, right) quadratic nodes; at 3/4 the mirror image.
    P = transfer.interpolation_1d(2, 2)
    assert np.allclose(P[1, :3], [3 / 8, 3 / 4, -1 / 8])
    assert np.allclose(P[3, :3], [-1 / 8, 3 / 4, 3 / 8])
    assert np.allclose(P[2, :3], [0, 1, 0])
    Q = transfer.interpolation_1d(2, 1)
    assert np.allclose(Q[1, :2], [0.5, 0.5])


@pytest.mark.parametrize("nc", [2, 4])
def test_galerkin_identity_on_free_dofs(nc):
    Af, _, dmf, _ = fem.stokes_system(2 * nc, 1.0)
    Ac, _, dmc, _ = fem.stokes_system(nc, 1.0)
    P = transfer.prolongation(nc)
    G = (P.T @ Af @ P).toarray()
    free = ~dmc
    diff = np.abs(G[np.ix_(free, free)] - Ac.toarray()[np.ix_(free, free)]).max()
    assert diff < 1e-13 * np.abs(Ac).max()


# ---------------------------------------------------------------- patches

def _table1(golden_dir):
    rows = {}
    with open(os.path.join(golden_dir, "table1_vanka_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, q, c0, c1, c2 = line.split()
            rows[(k, q)] = (int(c0), int(c1), int(c2))
    return rows


@pytest.mark.parametrize("N", [4, 7, 16])
def test_patch_sizes_match_table1(N, golden_dir):
    t1 = _table1(golden_dir)
    idx = vanka.patch_dofs(N)
    sizes = (idx >= 0).sum(axis=1)
    ell = N - 1

    def ev(key):
        c0, c1, c2 = t1[key]
        return c0 + c1 * ell + c2 * ell * ell

    assert sizes.sum() == ev(("form_patch_rhs", "reads"))
    assert sizes.sum() == ev(("update", "flops"))
    assert 2 * (sizes ** 2).sum() == ev(("apply_inverse", "flops"))
    assert (sizes ** 2 + sizes).sum() == ev(("apply_inverse", "reads"))
    assert sorted(set(sizes.tolist())) == [19, 31, 51]


@pytest.mark.parametrize("N", [8, 12])
def test_25_distinct_patch_matrices_and_exact_inverses(N):
    A, _, dmask, _ = fem.stokes_system(N, 1.0)
    idx = vanka.patch_dofs(N)
    keys = {}
    for k in range(idx.shape[0]):
        Ak = vanka.extract_patch_matrix(A, idx[k])
        key = (Ak.shape, Ak.tobytes(), tuple((idx[k] >= 0).tolist()))
        keys.setdefault(key, []).append(k)
        inv = np.linalg.inv(Ak)
        assert np.abs(Ak @ inv - np.eye(len(Ak))).max() < 1e-12
    # the paper: 25 patch matrices on a uniform mesh, independent of N;
    # 16 single patches, 8 edge strips, 1 interior region
    assert len(keys) == 25
    counts = sorted(len(v) for v in keys.values())
    assert counts[:16] == [1] * 16
    assert counts[16:24] == [N - 3] * 8
    assert counts[24] == (N - 3) ** 2
    # groups coincide with the distance classes
    cls = vanka.patch_classes(N)
    for members in keys.values():
        assert len(set(cls[members].tolist())) == 1


def test_multiplicities_on_free_dofs():
    N = 8
    g = grid_sizes(N)
    m = vanka.multiplicities(N)
    dmask = velocity_dirichlet_mask(N)
    s2 = g.q2_side
    for comp_off in (g.off_ux, g.off_uy):
        for j in range(1, s2 - 1):
            for i in range(1, s2 - 1):
                expect = {(0, 0): 9, (1, 0): 6, (0, 1): 6, (1, 1): 4}[(i % 2, j % 2)]
                assert m[comp_off + j * s2 + i] == expect
    assert np.all(m[g.off_p:] == 1)
    assert not np.any(m[~dmask] == 0)


def test_shared_inverses_equal_per_patch_inverses():
    N = 12
    A, b, dmask, _ = fem.stokes_system(N, 1.0)
    simple = vanka.VankaSmoother(A, N, dmask, 0.5, shared=False)
    tuned = vanka.VankaSmoother(A, N, dmask, 0.5, shared=True)
    for k in range(simple.inv.shape[0]):
        assert np.array_equal(simple.inv[k], tuned.inv[tuned.cls[k]])
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, A.shape[0])
    x[dmask] = 0
    # same operator; only the summation order of the batched products differs
    xs, xt = simple.sweep(x, b), tuned.sweep(x, b)
    assert np.abs(xs - xt).max() <= 1e-14 * np.abs(xs).max()


def test_vanka_sweep_matches_explicit_patch_loop():
    # Algorithm 3 written as a literal loop over patches on a tiny mesh.
    N = 4
    A, _, dmask, _ = fem.stokes_system(N, 1.0)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, A.shape[0])
    b = rng.uniform(-1, 1, A.shape[0])
    x[dmask] = 0
    b[dmask] = 0
    sm = vanka.VankaSmoother(A, N, dmask, 0.5, shared=False)
    r = b - A @ x
    m = np.zeros(A.shape[0])
    for k in range(sm.idx.shape[0]):
        for j in sm.idx[k][sm.idx[k] >= 0]:
            m[j] += 1
    upd = np.zeros_like(x)
    Ad = A.toarray()
    for k in range(sm.idx.shape[0]):
        S = sm.idx[k][sm.idx[k] >= 0]
        d = np.linalg.solve(Ad[np.ix_(S, S)], r[S])
        for jj, j in enumerate(S):
            if not dmask[j]:
                upd[j] += 0.5 / m[j] * d[jj]
    assert np.abs(sm.sweep(x, b) - (x + upd)).max() < 1e-12


# ---------------------------------------------------------------- V-cycle

def _vcycle_matrix(H):
    n = H.A.shape[0]
    return np.column_stack([H.vcycle(e) for e in np.eye(n)])


def test_vcycle_is_linear_and_contracts():
    N = 8
    H = multigrid.Hierarchy(N, 3)
    g = grid_sizes(N)
    rng = np.random.default_rng(3)
    dm = velocity_dirichlet_mask(N)
    u, v = rng.standard_normal(g.n), rng.standard_normal(g.n)
    u[dm] = v[dm] = 0
    assert np.allclose(H.vcycle(2 * u - 3 * v), 2 * H.vcycle(u) - 3 * H.vcycle(v), atol=1e-12)
    M = _vcycle_matrix(H)
    A = H.A.toarray()
    E = np.eye(g.n) - M @ A
    # error propagation on the free DoFs, modulo the pressure constant
    free = ~dm
    Q = np.eye(g.n)[:, free]
    c = np.zeros(g.n)
    c[g.off_p:] = 1.0
    c /= np.linalg.norm(c)
    Pi = np.eye(g.n) - np.outer(c, c)
    Ef = Q.T @ Pi @ E @ Pi @ Q
    rho = np.abs(np.linalg.eigvals(Ef)).max()
    # standalone V(2,2) contraction with omega = 0.5 and 1/m weights: 0.52
    assert rho < 0.6, rho


def test_coarse_bordered_solve_is_exact():
    N = 8
    H = multigrid.Hierarchy(N, 2)
    A0 = H.levels[0].A
    g0 = grid_sizes(H.levels[0].N)
    rng = np.random.default_rng(4)
    r = rng.standard_normal(A0.shape[0])
    r[velocity_dirichlet_mask(H.levels[0].N)] = 0
    r[g0.off_p:] -= r[g0.off_p:].mean()  # consistent
    e = H.coarse_solve(r)
    assert np.abs(A0 @ e - r).max() < 1e-11
    assert abs(e[g0.off_p:].sum()) < 1e-11


# ---------------------------------------------------------------- FGMRES

@pytest.mark.parametrize("N,levels", [(4, 2), (8, 2), (8, 3)])
def test_mg_fgmres_matches_dense_direct_solve(N, levels):
    H = multigrid.Hierarchy(N, levels)
    A, b, dm, xl = fem.stokes_system(N, 1.0, f_nodal=manufactured_nodal_force(N, "paper_poly"),
                                     g_nodal=manufactured_boundary_values(N, "paper_poly"))
    res = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-13, restart=30, max_iters=200)
    assert res.converged
    xd = direct_solve(N, A, b)
    xa = fem.normalise_pressure(N, res.x)
    xb = fem.normalise_pressure(N, xd)
    assert np.linalg.norm(xa - xb) <= 1e-10 * np.linalg.norm(xb)


def test_fgmres_iterate_minimises_residual_over_krylov_space():
    # With a fixed linear preconditioner M, FGMRES equals right-preconditioned
    # GMRES: after k steps x_k = x0 + M y with y in K_k(AM, r0) minimising
    # ||b - A x||.  Checked by brute-force least squares.
    N = 4
    H = multigrid.Hierarchy(N, 2)
    A, b, dm, xl = fem.stokes_system(N, 1.0, f_nodal=manufactured_nodal_force(N, "trig"))
    M = _vcycle_matrix(H)
    Ad = A.toarray()
    AM = Ad @ M
    r0 = b - Ad @ xl
    for k in range(1, 6):
        res = fgmres.fgmres(A, b, xl, H.vcycle, rtol=0.0, restart=30, fixed_iters=k)
        K = np.column_stack([np.linalg.matrix_power(AM, i) @ r0 for i in range(k)])
        Qk, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(AM @ Qk, r0, rcond=None)
        best = np.linalg.norm(r0 - AM @ Qk @ y)
        got = np.linalg.norm(b - Ad @ res.x)
        assert abs(got - best) <= 1e-9 * np.linalg.norm(r0) + 1e-6 * best


def test_fgmres_restart_and_edge_cases():
    N = 8
    H = multigrid.Hierarchy(N, 3)
    A, b, dm, xl = fem.stokes_system(N, 1.0, f_nodal=manufactured_nodal_force(N, "trig"))
    full = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8, restart=30)
    short = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8, restart=3)
    assert full.converged and short.converged
    assert short.restarts >= 1 and short.iterations >= full.iterations
    assert short.true_rel_res <= 1e-8
    # zero right-hand side: nothing to do
    z = fgmres.fgmres(A, np.zeros_like(b), np.zeros_like(b), H.vcycle)
    assert z.iterations == 0 and z.converged
    # iteration cap
    cap = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-14, max_iters=2)
    assert cap.iterations == 2 and not cap.converged


# ---------------------------------------------------------------- local forms

def test_residual_rows_match_assembled_operator():
    N = 8
    g = grid_sizes(N)
    A, _, dm, _ = fem.stokes_system(N, 1.0)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(g.n)
    b = rng.standard_normal(g.n)
    rows = np.arange(g.n)
    assert np.abs(fem.residual_rows(N, x, b, rows) - (b - A @ x)).max() < 1e-13


def test_local_patch_matrices_equal_extracted_blocks():
    N = 8
    A, _, _, _ = fem.stokes_system(N, 1.0)
    idx = vanka.patch_dofs(N)
    for k in range(idx.shape[0]):
        I, J = k % (N + 1), k // (N + 1)
        Al, S = vanka.local_patch_matrix(N, I, J)
        assert np.array_equal(S, idx[k][idx[k] >= 0])
        assert np.array_equal(Al, vanka.extract_patch_matrix(A, idx[k]))


def test_sampled_sweep_update_matches_full_sweep():
    N = 12
    A, _, dm, _ = fem.stokes_system(N, 1.0)
    g = grid_sizes(N)
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, g.n)
    b = rng.uniform(-1, 1, g.n)
    x[dm] = 0.0
    b[dm] = 0.0
    full = vanka.VankaSmoother(A, N, dm, 0.5, shared=False).sweep(x, b) - x
    dofs = np.concatenate([rng.choice(g.n, 60, replace=False),
                           [g.off_uy + 1 * g.q2_side + 1, g.off_p, g.off_p + g.n_pres - 1]])
    got = vanka.sampled_sweep_update(N, x, b, dofs)
    assert np.abs(got - full[dofs]).max() <= 1e-12 * np.abs(full).max()


def test_sampled_transfers_match_assembled_prolongation():
    nc = 6
    P = transfer.prolongation(nc)
    gf, gc = grid_sizes(2 * nc), grid_sizes(nc)
    rng = np.random.default_rng(8)
    ec = rng.standard_normal(gc.n)
    rf = rng.standard_normal(gf.n)
    assert np.abs(transfer.prolong_rows(nc, ec, np.arange(gf.n)) - P @ ec).max() < 1e-14
    assert np.abs(transfer.restrict_rows(nc, rf, np.arange(gc.n)) - P.T @ rf).max() < 1e-13
