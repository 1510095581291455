"""Pins of the oracle's inexact Braess-Sarazin relaxation (paper, section
"Braess-Sarazin relaxation scheme": the factorisation with L replaced by
t D, equations bseq1 / bseq2 and the algorithm).  Checked against a dense
solve of the approximate saddle-point system, the spectrum of the Schur
complement, and as a multigrid smoother."""

import numpy as np
import pytest

from oracle import fem, fgmres, multigrid
from oracle.braess_sarazin import BraessSarazinSmoother
from stokes_inputs import grid_sizes, uniform_vector, velocity_dirichlet_mask


def _residual(N, seed):
    g = grid_sizes(N)
    r = uniform_vector(g.n, seed)
    r[g.off_p:] -= r[g.off_p:].mean()  # consistent with the pressure null space of S
    return r


@pytest.mark.parametrize("t", [1.0, 1.7])
def test_exact_schur_step_solves_the_approximate_block_system(t):
    """With S inverted exactly, bseq1/bseq2 give the solution of
    [[t D, B^T], [B, 0]] [du; dp] = r (D = diagonal of the velocity block),
    built here from the assembled operator."""
    N = 4
    A, _, _, _ = fem.stokes_system(N)
    g = grid_sizes(N)
    nv = g.off_p
    Ad = A.toarray()
    D = np.diag(np.diag(Ad[:nv, :nv]))
    K = np.zeros_like(Ad)
    K[:nv, :nv] = t * D
    K[:nv, nv:] = Ad[:nv, nv:]
    K[nv:, :nv] = Ad[nv:, :nv]
    r = _residual(N, 31)
    sol = np.linalg.lstsq(K, r, rcond=None)[0]
    sm = BraessSarazinSmoother(A, N, t=t)
    rhs = sm.schur_rhs(r)
    dp = np.linalg.lstsq(sm.S.toarray(), rhs, rcond=None)[0]
    du = (1.0 / t) * sm.Dinv * (r[:nv] - sm.BT @ dp)
    assert np.allclose(du, sol[:nv], rtol=0, atol=1e-10 * np.abs(sol[:nv]).max())
    dps, dpk = dp - dp.mean(), sol[nv:] - sol[nv:].mean()
    assert np.allclose(dps, dpk, rtol=0, atol=1e-10 * np.abs(dpk).max())
    # and K [du; dp] = r
    assert np.allclose(K @ np.concatenate([du, dp]), r, atol=1e-10 * np.abs(r).max())


def test_schur_complement_is_negative_semidefinite_with_constant_null_space():
    N = 4
    A, _, _, _ = fem.stokes_system(N)
    sm = BraessSarazinSmoother(A, N, t=1.3)
    S = sm.S.toarray()
    assert np.allclose(S, S.T, atol=1e-15)
    w, V = np.linalg.eigh(S)
    assert w.max() < 1e-14 * abs(w.min())
    assert np.sum(np.abs(w) < 1e-12 * abs(w.min())) == 1
    v0 = V[:, np.argmax(w)]
    assert np.allclose(np.abs(v0), np.abs(v0).mean(), atol=1e-10)
    assert np.allclose(np.diag(S), sm.Sdiag)


def test_jacobi_sweeps_converge_to_the_exact_schur_step():
    N = 4
    A, _, _, _ = fem.stokes_system(N)
    r = _residual(N, 32)
    exact = BraessSarazinSmoother(A, N, t=1.0)
    dp_ex = np.linalg.lstsq(exact.S.toarray(), exact.schur_rhs(r), rcond=None)[0]
    dp_ex -= dp_ex.mean()
    sm = BraessSarazinSmoother(A, N, t=1.0, jacobi_weight=0.6, jacobi_sweeps=3000)
    c = sm.correction(r)
    nv = sm.nv
    dp = c[nv:] - c[nv:].mean()
    assert np.linalg.norm(dp - dp_ex) <= 1e-8 * np.linalg.norm(dp_ex)
    # one sweep from zero is the weighted diagonal solve
    one = BraessSarazinSmoother(A, N, t=1.0, jacobi_weight=0.7, jacobi_sweeps=1)
    rhs = one.schur_rhs(r)
    assert np.allclose(one.correction(r)[nv:], 0.7 * rhs / np.diag(one.S.toarray()))


def test_dirichlet_rows_get_the_scaled_residual():
    N = 4
    A, _, _, _ = fem.stokes_system(N)
    r = _residual(N, 33)
    sm = BraessSarazinSmoother(A, N, t=2.0)
    c = sm.correction(r)
    m = velocity_dirichlet_mask(N)[:sm.nv]
    assert np.allclose(c[:sm.nv][m], r[:sm.nv][m] / 2.0)


def test_braess_sarazin_multigrid_contracts_and_solves():
    N, levels = 16, 3
    H = multigrid.Hierarchy(N, levels, relaxation="bs")
    A = H.A
    n = A.shape[0]
    off_p = grid_sizes(N).off_p
    dm = velocity_dirichlet_mask(N)
    rng = np.random.default_rng(5)
    e = rng.standard_normal(n)
    e[dm] = 0.0
    for _ in range(10):
        e2 = e - H.vcycle(A @ e)
        e2[off_p:] -= e2[off_p:].mean()
        rho = np.linalg.norm(e2) / np.linalg.norm(e)
        e = e2 / np.linalg.norm(e2)
    assert rho < 0.2
    # FGMRES with the Braess-Sarazin V-cycle reaches the dense solution
    x_true = rng.standard_normal(n)
    x_true[dm] = 0.0
    x_true[off_p:] -= x_true[off_p:].mean()
    b = A @ x_true
    res = fgmres.fgmres(A, b, np.zeros(n), H.vcycle, rtol=1e-10, restart=30, max_iters=60)
    assert res.converged
    xs = res.x.copy()
    xs[off_p:] -= xs[off_p:].mean()
    assert np.linalg.norm(xs - x_true) <= 1e-8 * np.linalg.norm(x_true)
