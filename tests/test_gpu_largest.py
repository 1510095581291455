"""GPU checks at 4096 x 4096 elements (10 levels, 151 M unknowns, a Krylov
basis of ~75 GB): the largest mesh of this family that leaves room on one
GPU, four times the benchmark's side.  The launches there exceed 65535
workgroups per grid dimension and every per-level vector exceeds 1 GB.

As at 1024 x 1024, local steps are compared with the oracle at sampled
outputs (residual rows, Vanka updates), global ones through properties that
hold at any size (linearity and contraction of the V-cycle, FGMRES reaching
the requested true residual, checked again at sampled rows).
"""

import numpy as np
import pytest

from oracle import fem, vanka
from stokes_inputs import (dirichlet_consistent_pair, grid_sizes, uniform_vector,
                           velocity_dirichlet_mask)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2401_06277_amd as vk  # noqa: E402

N_MAX, LEVELS_MAX = 4096, 10


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def note(msg):
    print(msg, flush=True)


def close(got, want, tol):
    scale = max(np.abs(want).max(), 1e-300)
    err = np.abs(got - want).max() / scale
    assert err <= tol, f"max rel err {err:.3e} > {tol:g}"


def sample_dofs(N, seed, n_random=60):
    """Corners, edges, tile seams of the Vanka (14 elements) and residual (16
    elements) kernels at the far end of the mesh, and random DoFs."""
    g = grid_sizes(N)
    s2, s1 = g.q2_side, g.q1_side
    near = [0, 1, 2, 3, 5, s2 // 2, s2 - 30, s2 - 29, s2 - 6, s2 - 3, s2 - 2, s2 - 1]
    dofs = []
    for k, qi in enumerate(near):
        qj = near[(5 * k + 3) % len(near)]
        dofs += [g.off_ux + qj * s2 + qi, g.off_uy + qi * s2 + qj]
    for I, J in [(0, 0), (1, s1 - 2), (s1 - 1, 2), (s1 // 2, s1 - 1), (s1 - 15, s1 - 14)]:
        dofs.append(g.off_p + J * s1 + I)
    rng = np.random.default_rng(seed)
    dofs += list(rng.choice(g.n, n_random, replace=False))
    return np.array(sorted(set(int(d) for d in dofs)))


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    note(f"setup N={N_MAX} levels={LEVELS_MAX}")
    s = vk.VkmgSolver(N_MAX, LEVELS_MAX)
    note("inputs")
    x, b = dirichlet_consistent_pair(N_MAX, 201, 202)
    yield s, x, b
    s.close()
    torch.cuda.empty_cache()


def test_largest_residual_sampled_rows(ctx):
    s, x, b = ctx
    rows = sample_dofs(N_MAX, 203)
    note(f"residual: {len(rows)} sampled rows")
    r = host(s.residual(dev(b), dev(x)))
    close(r[rows], fem.residual_rows(N_MAX, x, b, rows), 1e-13)


def test_largest_vanka_sweep_sampled(ctx):
    s, x, b = ctx
    dofs = sample_dofs(N_MAX, 204)
    note(f"vanka sweep: {len(dofs)} sampled DoFs")
    xg = dev(x)
    s.vanka_sweep(LEVELS_MAX - 1, xg, dev(b))
    xn = host(xg)
    got = xn[dofs] - x[dofs]
    want = vanka.sampled_sweep_update(N_MAX, x, b, dofs)
    vel = dofs < grid_sizes(N_MAX).off_p
    close(got[vel], want[vel], 1e-12)
    close(got[~vel], want[~vel], 1e-12)
    dm = velocity_dirichlet_mask(N_MAX)
    assert np.array_equal(xn[dm], x[dm])


def test_largest_vcycle_linear_and_contracting(ctx):
    s, _, _ = ctx
    g = grid_sizes(N_MAX)
    mask = dev(velocity_dirichlet_mask(N_MAX))
    r = dev(uniform_vector(g.n, 205))
    r[mask] = 0.0
    z = s.vcycle(r)
    z2 = s.vcycle(2.5 * r)
    err = float(torch.linalg.vector_norm(z2 - 2.5 * z) / torch.linalg.vector_norm(2.5 * z))
    note(f"V-cycle linearity {err:.2e}")
    assert err <= 1e-12
    del z, z2
    e = dev(uniform_vector(g.n, 206))
    e[mask] = 0.0
    norms = []
    for _ in range(12):
        e = e - s.vcycle(s.apply(e))
        e[g.off_p:] -= e[g.off_p:].mean()
        norms.append(float(torch.linalg.vector_norm(e)))
    rate = (norms[-1] / norms[5]) ** (1.0 / 6)
    note(f"V-cycle error contraction at N={N_MAX}: {rate:.3f} per cycle")
    assert rate < 0.6


def test_largest_fgmres_solve(ctx):
    s, _, _ = ctx
    g = grid_sizes(N_MAX)
    f = uniform_vector(2 * g.q2_side ** 2, 207)
    b = s.assemble_rhs(dev(f))
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    info = s.fgmres_solve(b, x, rtol=1e-8, restart=30, max_iters=200)
    note(f"fgmres N={N_MAX}: {info}")
    assert info["status_name"] == "VKMG_OK"
    assert info["true_rel_res"] <= 1e-8 and info["iterations"] <= 40
    bh, xh = host(b), host(x)
    rows = sample_dofs(N_MAX, 208, 200)
    assert np.abs(fem.residual_rows(N_MAX, xh, bh, rows)).max() <= 1e-8 * np.linalg.norm(bh)
