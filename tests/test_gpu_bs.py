"""GPU parity of the Braess-Sarazin relaxation (vkmg_relax on a context
with relaxation = VKMG_RELAX_BRAESS_SARAZIN) against the oracle's
BraessSarazinSmoother on the same seeded inputs.  Tolerances as for Vanka:
one relaxation on every level 1e-12 (FP64) / 1e-5 (FP32), V-cycle 1e-11,
FGMRES iterations +-1 at rtol 1e-8 and the solution at equal iteration
counts 1e-10; every error is taken per field (u_x, u_y, p, each against
its own magnitude)."""

import numpy as np
import pytest

from oracle import fem, fgmres, multigrid
from oracle.braess_sarazin import BraessSarazinSmoother
from stokes_inputs import (manufactured_boundary_values, manufactured_nodal_force,
                           uniform_vector, velocity_dirichlet_mask)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2401_06277_amd as vk  # noqa: E402
from fieldwise import rel, rel2  # noqa: E402  (each field against its own magnitude)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


PARAMS = [dict(t=1.0, omega_bs=1.0, jacobi_weight=1.0, jacobi_sweeps=2),
          dict(t=1.3, omega_bs=0.8, jacobi_weight=0.7, jacobi_sweeps=1),
          dict(t=1.1, omega_bs=0.9, jacobi_weight=0.9, jacobi_sweeps=3)]


def _solver(N, levels, p, precision="fp64", batch=1):
    return vk.VkmgSolver(N, levels, precision=precision, relaxation="braess_sarazin",
                         bs_t=p["t"], bs_omega=p["omega_bs"], bs_jacobi_weight=p["jacobi_weight"],
                         bs_jacobi_sweeps=p["jacobi_sweeps"], batch=batch)


@pytest.mark.parametrize("pi", range(len(PARAMS)))
@pytest.mark.parametrize("N,levels", [(16, 3), (24, 3), (40, 3)])
def test_bs_relaxation_every_level(N, levels, pi):
    p = PARAMS[pi]
    note(f"bs relax N={N} params={p}")
    s = _solver(N, levels, p)
    for level in range(1, levels):
        Nl = N >> (levels - 1 - level)
        A, _, _, _ = fem.stokes_system(Nl)
        sm = BraessSarazinSmoother(A, Nl, **p)
        n = A.shape[0]
        x = uniform_vector(n, 40 + level)
        b = uniform_vector(n, 50 + level)
        xg = dev(x)
        s.relax(level, xg, dev(b))
        assert rel(host(xg), sm.sweep(x, b)) < 1e-12, level
    s.close()


def test_bs_relaxation_fp32():
    p = PARAMS[0]
    N, levels = 24, 3
    s = _solver(N, levels, p, precision="fp32")
    A, _, _, _ = fem.stokes_system(N)
    sm = BraessSarazinSmoother(A, N, **p)
    n = A.shape[0]
    x = uniform_vector(n, 61)
    b = uniform_vector(n, 62)
    xg = dev(x, torch.float32)
    s.relax(levels - 1, xg, dev(b, torch.float32))
    assert rel(host(xg), sm.sweep(x.astype(np.float32).astype(np.float64),
                                  b.astype(np.float32).astype(np.float64))) < 1e-5
    s.close()


@pytest.mark.parametrize("N,levels", [(16, 3), (32, 4), (48, 3)])
def test_bs_vcycle(N, levels):
    note(f"bs vcycle N={N}")
    p = PARAMS[0]
    s = _solver(N, levels, p)
    H = multigrid.Hierarchy(N, levels, relaxation="bs", bs=p)
    n = H.A.shape[0]
    r = uniform_vector(n, 70)
    r[velocity_dirichlet_mask(N)] = 0.0
    z = host(s.vcycle(dev(r)))
    assert rel(z, H.vcycle(r)) < 1e-11
    s.close()


@pytest.mark.parametrize("N,levels", [(16, 3), (32, 4)])
def test_bs_fgmres_iterations_and_solution(N, levels):
    note(f"bs fgmres N={N}")
    p = PARAMS[0]
    s = _solver(N, levels, p)
    H = multigrid.Hierarchy(N, levels, relaxation="bs", bs=p)
    gd = manufactured_boundary_values(N, "trig")
    A, b, _, xl = fem.stokes_system(N, 1.0, f_nodal=manufactured_nodal_force(N, "trig"),
                                    g_nodal=gd)
    ro = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8, restart=30, max_iters=200)
    x = dev(xl)
    info = s.fgmres_solve(dev(b), x, rtol=1e-8, restart=30, max_iters=200)
    assert info["status_name"] == "VKMG_OK"
    assert abs(info["iterations"] - ro.iterations) <= 1
    k = ro.iterations
    x = dev(xl)
    info_k = s.fgmres_solve(dev(b), x, rtol=0.0, restart=30, max_iters=k)
    assert info_k["iterations"] == k
    ok = fgmres.fgmres(A, b, xl, H.vcycle, rtol=0.0, restart=30, fixed_iters=k)
    xa = fem.normalise_pressure(N, host(x))
    xo = fem.normalise_pressure(N, ok.x)
    assert rel2(xa, xo) <= 1e-10
    s.close()


def test_bs_batched_vcycle_equals_single_bitwise():
    p = PARAMS[2]
    N, levels, B = 24, 3, 3
    sb = _solver(N, levels, p, batch=B)
    s1 = _solver(N, levels, p)
    n = s1.layout["n"]
    rs = [uniform_vector(n, 80 + k) for k in range(B)]
    zb = host(sb.vcycle(dev(np.concatenate(rs)))).reshape(B, n)
    for k in range(B):
        assert np.array_equal(zb[k], host(s1.vcycle(dev(rs[k]))))
    sb.close()
    s1.close()


def test_bs_fp32_multigrid_fgmres_reaches_fp64_tolerance():
    N, levels = 32, 4
    s = _solver(N, levels, PARAMS[0], precision="fp32")
    gd = manufactured_boundary_values(N, "trig")
    A, b, _, xl = fem.stokes_system(N, 1.0, f_nodal=manufactured_nodal_force(N, "trig"),
                                    g_nodal=gd)
    x = dev(xl)
    info = s.fgmres_solve(dev(b), x, rtol=1e-8, restart=30, max_iters=200)
    assert info["status_name"] == "VKMG_OK"
    assert np.linalg.norm(b - A @ host(x)) <= 1.01e-8 * np.linalg.norm(b - A @ xl)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bs_benchmark_solve_matches_oracle_golden(precision):
    """The benchmark's Braess-Sarazin solve at 1024 x 1024, 8 levels (GRF
    force seed 5, x0 = 0, t = 1, omega_BS = 1, two Jacobi sweeps of weight 1,
    FGMRES(30) to 1e-8) against the oracle's (tests/golden/bs_oracle_1024.json,
    written by tests/golden/make_bs_oracle.py): iteration count within one;
    after exactly the oracle's count, with the V-cycle in FP64 the solution
    within 1e-10 of each field's maximum at the sampled DoFs and the true
    relative residual equal to the oracle's to 1e-3 relative; with the
    V-cycle in FP32 (FGMRES in FP64) the true relative residual at the
    tolerance and the solution within 1e-8 per field (the FP32 cycle changes
    the Krylov path, so the solves agree to their distance from the exact
    solution, not to rounding)."""
    import json
    import os

    from stokes_inputs import gaussian_random_field, grid_sizes
    N, levels = 1024, 8
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bs_oracle_1024.json")
    with open(path) as fh:
        d = json.load(fh)
    assert d["N"] == N and d["levels"] == levels and d["bs"] == PARAMS[0]
    note(f"[BS golden] N={N} levels={levels} {precision}")
    gs = grid_sizes(N)
    dofs = np.array(d["dofs"])
    field = np.searchsorted([gs.off_uy, gs.off_p], dofs, side="right")
    s = _solver(N, levels, PARAMS[0], precision=precision)
    b = s.assemble_rhs(dev(gaussian_random_field(N, 5, length=0.1).ravel()))
    x = torch.zeros_like(b)
    info = s.fgmres_solve(b, x, rtol=1e-8, restart=30, max_iters=200)
    note(f"[BS golden] GPU {info['iterations']} iterations, oracle {d['iterations']}")
    assert info["status_name"] == "VKMG_OK"
    assert abs(info["iterations"] - d["iterations"]) <= 1
    m = d["iterations"]
    x = torch.zeros_like(b)
    info_m = s.fgmres_solve(b, x, rtol=0.0, restart=30, max_iters=m)
    assert info_m["iterations"] == m
    if precision == "fp64":
        assert abs(info_m["true_rel_res"] - d["true_rel_res"]) <= 1e-3 * d["true_rel_res"]
    else:
        assert info_m["true_rel_res"] <= 1e-8, info_m
    xn = fem.normalise_pressure(N, host(x))
    want = np.array(d["solution"])
    worst = []
    for f in range(3):
        sel = field == f
        assert sel.sum() > 1000
        worst.append(float(np.abs(xn[dofs][sel] - want[sel]).max() / d["solution_field_max"][f]))
    note(f"[BS golden] after {m} steps ({precision} V-cycle): per-field max error "
         f"{['%.2e' % e for e in worst]}, true rel res {info_m['true_rel_res']:.2e}")
    assert max(worst) <= (1e-10 if precision == "fp64" else 1e-8), worst
    s.close()
