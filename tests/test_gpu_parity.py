"""GPU parity: every step of the hot path through the C ABI against the CPU
oracle on the same seeded inputs (small meshes spanning several tiles and
ragged tails).  Tolerances (relative, FP64 path):
(each of u_x, u_y and p against its own magnitude: after a sweep or a
V-cycle the pressure is ~1/h^2 larger than the velocity)
  residual / operator apply / right-hand side / transfers   1e-13
  one Vanka sweep                                          1e-12
  coarse solve, V-cycle application                         1e-11
  FGMRES solution at an equal iteration count               1e-10
  FGMRES iteration count at rtol 1e-8                       +-1
The FP32 multigrid path is compared with the FP64 oracle at 1e-5
(single-precision rounding of O(1) data through a few operations).
"""

import numpy as np
import pytest

from oracle import fem, fgmres, multigrid, transfer, vanka
from stokes_inputs import (dirichlet_consistent_pair, gaussian_random_field, grid_sizes,
                           manufactured_boundary_values, manufactured_nodal_force,
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


_solvers = {}


def solver(N, levels, precision="fp64", apply="vector"):
    key = (N, levels, precision, apply)
    if key not in _solvers:
        _solvers[key] = vk.VkmgSolver(N, levels, precision=precision, interior_apply=apply)
    return _solvers[key]


_hier = {}


def hierarchy(N, levels):
    key = (N, levels)
    if key not in _hier:
        _hier[key] = multigrid.Hierarchy(N, levels)
    return _hier[key]


MESHES = [(4, 2), (16, 3), (24, 3), (32, 4), (40, 3)]


@pytest.mark.parametrize("N,levels", MESHES)
def test_residual_and_apply(N, levels):
    note(f"residual N={N}")
    s = solver(N, levels)
    A = hierarchy(N, levels).A
    g = grid_sizes(N)
    x = uniform_vector(g.n, 11)
    b = uniform_vector(g.n, 12)
    r = host(s.residual(dev(b), dev(x)))
    ro = b - A @ x
    assert rel(r, ro) < 1e-13
    y = host(s.apply(dev(x)))
    assert rel(y, A @ x) < 1e-13


@pytest.mark.parametrize("N", [8, 24])
def test_assemble_rhs(N):
    note(f"rhs N={N}")
    s = solver(N, 2 if N == 8 else 3)
    f = gaussian_random_field(N, 21, length=0.2)
    gd = manufactured_boundary_values(N, "paper_poly")
    _, b_o, _, _ = fem.stokes_system(N, 1.0, f_nodal=f, g_nodal=gd)
    b = host(s.assemble_rhs(dev(f.ravel()), dev(gd.ravel())))
    assert rel(b, b_o) < 1e-13
    _, b_o0, _, _ = fem.stokes_system(N, 1.0, f_nodal=f)
    b0 = host(s.assemble_rhs(dev(f.ravel())))
    assert rel(b0, b_o0) < 1e-13


@pytest.mark.parametrize("N,levels", MESHES)
def test_vanka_sweep_every_level(N, levels):
    s = solver(N, levels)
    H = hierarchy(N, levels)
    for l in range(1, levels):
        lev = H.levels[l]
        note(f"vanka N={N} level={l} (N_l={lev.N})")
        x, b = dirichlet_consistent_pair(lev.N, 30 + l, 40 + l)
        xg = dev(x)
        s.vanka_sweep(l, xg, dev(b))
        xo = lev.smoother.sweep(x, b)
        assert rel(host(xg), xo) < 1e-12
        # two sweeps in a row (the updated x feeds the next residual)
        s.vanka_sweep(l, xg, dev(b))
        assert rel(host(xg), lev.smoother.sweep(xo, b)) < 1e-12


@pytest.mark.parametrize("omega", [0.3, 0.75, 1.0])
def test_vanka_sweep_other_damping(omega):
    """The damping enters both the boundary-class tables and the scaled
    interior constants; a sweep on every level with omega != 0.5 and the
    V-cycle against the oracle built with the same omega."""
    N, levels = 24, 3
    s = vk.VkmgSolver(N, levels, omega=omega)
    H = multigrid.Hierarchy(N, levels, omega=omega)
    for l in range(1, levels):
        lev = H.levels[l]
        x, b = dirichlet_consistent_pair(lev.N, 60 + l, 70 + l)
        xg = dev(x)
        s.vanka_sweep(l, xg, dev(b))
        assert rel(host(xg), lev.smoother.sweep(x, b)) < 1e-12
    r = uniform_vector(H.A.shape[0], 77)
    r[velocity_dirichlet_mask(N)] = 0.0
    assert rel(host(s.vcycle(dev(r))), H.vcycle(r)) < 1e-11
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_interior_apply_variants_agree(precision, tol):
    """The matrix-instruction and vector-ALU interior applies against the
    oracle, on every relaxed level of a mesh with several tiles."""
    N, levels = 40, 3
    H = hierarchy(N, levels)
    dt = torch.float32 if precision == "fp32" else torch.float64
    for apply in ("matrix", "vector"):
        s = solver(N, levels, precision, apply)
        for l in range(1, levels):
            lev = H.levels[l]
            note(f"{apply} {precision} sweep level={l}")
            x, b = dirichlet_consistent_pair(lev.N, 130 + l, 140 + l)
            xg = dev(x, dt)
            s.vanka_sweep(l, xg, dev(b, dt))
            if precision == "fp32":
                x = x.astype(np.float32).astype(np.float64)
                b = b.astype(np.float32).astype(np.float64)
            assert rel(host(xg), lev.smoother.sweep(x, b)) < tol


@pytest.mark.parametrize("apply", ["vector", "matrix"])
def test_vanka_update_given_residual(apply):
    """The update half of a sweep: x + S (b - A x) with the residual formed
    by the oracle equals the oracle sweep."""
    N, levels = 40, 3
    s = solver(N, levels, apply=apply)
    H = hierarchy(N, levels)
    lev = H.levels[-1]
    x, b = dirichlet_consistent_pair(N, 160, 161)
    r = b - lev.A @ x
    xg = dev(x)
    s.vanka_update(levels - 1, xg, dev(r))
    assert rel(host(xg), lev.smoother.sweep(x, b)) < 1e-12
    with pytest.raises(vk.VkmgError):
        s.vanka_update(levels - 1, xg, xg)


def test_vanka_sweep_is_bitwise_reproducible():
    s = solver(40, 3)
    x, b = dirichlet_consistent_pair(40, 5, 6)
    outs = []
    for _ in range(2):
        xg = dev(x)
        s.vanka_sweep(2, xg, dev(b))
        outs.append(host(xg))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("N,levels", MESHES)
def test_transfers(N, levels):
    s = solver(N, levels)
    for l in range(1, levels):
        note(f"transfer N={N} level={l}")
        Nf = N >> (levels - 1 - l)
        P = transfer.prolongation(Nf // 2)
        gf, gc = grid_sizes(Nf), grid_sizes(Nf // 2)
        rf = uniform_vector(gf.n, 50 + l)
        bc = host(s.restrict(l, dev(rf)))
        assert rel(bc, P.T @ rf) < 1e-13
        ec = uniform_vector(gc.n, 60 + l)
        ec[velocity_dirichlet_mask(Nf // 2)] = 0.0
        xf = uniform_vector(gf.n, 70 + l)
        xg = dev(xf)
        s.prolong_add(l, dev(ec), xg)
        assert rel(host(xg), xf + P @ ec) < 1e-13


@pytest.mark.parametrize("N,levels", [(16, 3), (32, 3), (64, 4)])
def test_coarse_solve(N, levels):
    note(f"coarse N={N}")
    s = solver(N, levels)
    H = hierarchy(N, levels)
    n0 = H.levels[0].n
    r = uniform_vector(n0, 80)
    r[velocity_dirichlet_mask(H.levels[0].N)] = 0.0
    e = host(s.coarse_solve(dev(r)))
    assert rel(e, H.coarse_solve(r)) < 1e-11


@pytest.mark.parametrize("N,levels", [(16, 3), (24, 3), (32, 4), (48, 3)])
def test_vcycle(N, levels):
    note(f"vcycle N={N} levels={levels}")
    s = solver(N, levels)
    H = hierarchy(N, levels)
    g = grid_sizes(N)
    r = uniform_vector(g.n, 90)
    r[velocity_dirichlet_mask(N)] = 0.0
    z = host(s.vcycle(dev(r)))
    assert rel(z, H.vcycle(r)) < 1e-11


@pytest.mark.parametrize("nu_pre,nu_post", [(1, 1), (1, 2), (0, 2), (3, 0), (0, 0), (2, 3)])
def test_vcycle_shapes(nu_pre, nu_post):
    # odd sweep counts exercise the alternation of the fused sweeps' buffers
    N, levels = 32, 3
    note(f"vcycle V({nu_pre},{nu_post})")
    s = vk.VkmgSolver(N, levels, nu_pre=nu_pre, nu_post=nu_post)
    H = multigrid.Hierarchy(N, levels, nu_pre=nu_pre, nu_post=nu_post)
    g = grid_sizes(N)
    r = uniform_vector(g.n, 91)
    r[velocity_dirichlet_mask(N)] = 0.0
    z = host(s.vcycle(dev(r)))
    assert rel(z, H.vcycle(r)) < 1e-11
    s.close()


def _manufactured_system(N, name="trig"):
    gd = manufactured_boundary_values(N, name)
    A, b, dm, xl = fem.stokes_system(N, 1.0, f_nodal=manufactured_nodal_force(N, name), g_nodal=gd)
    return A, b, xl, gd


@pytest.mark.parametrize("N,levels,name", [(16, 3, "trig"), (32, 4, "paper_poly"), (40, 3, "trig")])
def test_fgmres_iterations_and_solution(N, levels, name):
    note(f"fgmres N={N} levels={levels} {name}")
    s = solver(N, levels)
    H = hierarchy(N, levels)
    A, b, xl, gd = _manufactured_system(N, name)
    ro = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8, restart=30, max_iters=500)
    x = dev(xl)
    info = s.fgmres_solve(dev(b), x, rtol=1e-8, restart=30, max_iters=500)
    assert info["status_name"] == "VKMG_OK"
    assert abs(info["iterations"] - ro.iterations) <= 1
    assert info["true_rel_res"] <= 1e-8
    # equal iteration counts: GPU with rtol 0 and a cap, oracle with fixed_iters
    k = ro.iterations
    x = dev(xl)
    info_k = s.fgmres_solve(dev(b), x, rtol=0.0, restart=30, max_iters=k)
    assert info_k["iterations"] == k
    ok = fgmres.fgmres(A, b, xl, H.vcycle, rtol=0.0, restart=30, fixed_iters=k)
    xa = fem.normalise_pressure(N, host(x))
    xo = fem.normalise_pressure(N, ok.x)
    assert rel2(xa, xo) <= 1e-10



@pytest.mark.parametrize("N,levels", [(24, 3), (32, 4)])
def test_fgmres_long_restart_matches_oracle(N, levels):
    """The classical CGS2 path (restart lengths above 32, host rotations) at
    equal iteration counts, on larger meshes than the test below: FGMRES(40)
    against the oracle's FGMRES(40), iteration count within one at rtol 1e-10
    and, after exactly the oracle's count, the solution within 1e-10."""
    note(f"fgmres restart 40 N={N} levels={levels}")
    s = solver(N, levels)
    H = hierarchy(N, levels)
    A, b, xl, _ = _manufactured_system(N, "trig")
    ro = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-10, restart=40, max_iters=500)
    x = dev(xl)
    info = s.fgmres_solve(dev(b), x, rtol=1e-10, restart=40, max_iters=500)
    assert info["status_name"] == "VKMG_OK"
    assert abs(info["iterations"] - ro.iterations) <= 1
    assert info["true_rel_res"] <= 1e-10
    k = ro.iterations
    x = dev(xl)
    info_k = s.fgmres_solve(dev(b), x, rtol=0.0, restart=40, max_iters=k)
    assert info_k["iterations"] == k
    ok = fgmres.fgmres(A, b, xl, H.vcycle, rtol=0.0, restart=40, fixed_iters=k)
    xa = fem.normalise_pressure(N, host(x))
    xo = fem.normalise_pressure(N, ok.x)
    err = rel2(xa, xo)
    note(f"  {k} iterations, solution difference {err:.2e}")
    assert err <= 1e-10

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fgmres_graph_replays_match_direct_launches(precision):
    """Each Arnoldi step replayed as a captured graph gives bitwise the same
    iterates as direct launches, across replays separated by eager work,
    restart lengths that reallocate the basis (recapture) and steps beyond
    32 basis vectors (unfused Gram-Schmidt)."""
    N, levels = 32, 4
    sg = vk.VkmgSolver(N, levels, precision=precision, graphs=True)
    sd = vk.VkmgSolver(N, levels, precision=precision, graphs=False)
    _, b, xl, _ = _manufactured_system(N)
    bg = dev(b)
    for rtol, restart, iters in [(1e-10, 8, 200), (0.0, 40, 36), (1e-10, 8, 200), (1e-10, 8, 200)]:
        note(f"graphs {precision} rtol={rtol} restart={restart}")
        xg, xd = dev(xl), dev(xl)
        ig = sg.fgmres_solve(bg, xg, rtol=rtol, restart=restart, max_iters=iters)
        idr = sd.fgmres_solve(bg, xd, rtol=rtol, restart=restart, max_iters=iters)
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda", dtype=torch.float64)
        assert float((junk * junk).sum()) > 0.0
        assert ig["iterations"] == idr["iterations"] and ig["restarts"] == idr["restarts"]
        assert torch.equal(xg, xd)
    # kernel timing inside graphs counts every replayed Vanka update
    for s in (sg, sd):
        s.set_timing(1 << vk.KERNEL_VANKA)
        x = dev(xl)
        info = s.fgmres_solve(bg, x, rtol=1e-10, restart=8, max_iters=200)
        n, ms = s.kernel_timing(vk.KERNEL_VANKA, levels - 1)
        s.set_timing(0)
        assert n == 4 * info["iterations"] and ms > 0.0
    sg.close()
    sd.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fgmres_pipelined_steps_stop_where_direct_launches_do(precision):
    """With graphs the next Arnoldi step is enqueued before the host has
    tested the current one (unless convergence is predicted).  Across
    tolerances that stop the solve at different steps of a cycle, short
    restarts, an iteration cap and a fixed iteration count, the iteration
    counts, statuses and iterates equal those of direct launches (which never
    run ahead)."""
    N, levels = 32, 4
    sg = vk.VkmgSolver(N, levels, precision=precision, graphs=True)
    sd = vk.VkmgSolver(N, levels, precision=precision, graphs=False)
    _, b, xl, _ = _manufactured_system(N)
    bg = dev(b)
    cases = [(rt, 30, 200) for rt in (1e-1, 3e-3, 1e-4, 2e-6, 1e-8, 5e-10, 1e-11)]
    cases += [(1e-9, 3, 200), (1e-9, 5, 200), (1e-12, 30, 7), (0.0, 30, 9)]
    for rtol, restart, iters in cases:
        note(f"pipelined {precision} rtol={rtol} restart={restart} max_iters={iters}")
        xg, xd = dev(xl), dev(xl)
        ig = sg.fgmres_solve(bg, xg, rtol=rtol, restart=restart, max_iters=iters)
        idr = sd.fgmres_solve(bg, xd, rtol=rtol, restart=restart, max_iters=iters)
        assert (ig["iterations"], ig["restarts"], ig["status_name"]) == \
            (idr["iterations"], idr["restarts"], idr["status_name"])
        assert ig["true_rel_res"] == idr["true_rel_res"]
        assert torch.equal(xg, xd)
    sg.close()
    sd.close()


def test_fgmres_restarts_match_oracle():
    N, levels = 16, 3
    s = solver(N, levels)
    H = hierarchy(N, levels)
    A, b, xl, _ = _manufactured_system(N)
    ro = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-10, restart=4, max_iters=200)
    x = dev(xl)
    info = s.fgmres_solve(dev(b), x, rtol=1e-10, restart=4, max_iters=200)
    assert info["status_name"] == "VKMG_OK"
    assert abs(info["iterations"] - ro.iterations) <= 1
    assert info["restarts"] >= 1
    xa = fem.normalise_pressure(N, host(x))
    xo = fem.normalise_pressure(N, ro.x)
    assert rel2(xa, xo) <= 1e-8


def test_fgmres_long_restart_classical_path():
    """Restarts above 32 use the classical three-pass CGS2 (unfused passes
    beyond 32 basis vectors, the new vector scaled on host request): the
    iteration count and solution at rtol 1e-10 match the oracle, and 36
    steps of one cycle (rtol 0, more than 32 basis vectors) reach the
    rounding floor with the oracle's solution."""
    N, levels = 16, 3
    s = solver(N, levels)
    H = hierarchy(N, levels)
    A, b, xl, _ = _manufactured_system(N)
    ro = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-10, restart=40, max_iters=200)
    x = dev(xl)
    info = s.fgmres_solve(dev(b), x, rtol=1e-10, restart=40, max_iters=200)
    assert info["status_name"] == "VKMG_OK"
    assert abs(info["iterations"] - ro.iterations) <= 1
    xo = fem.normalise_pressure(N, ro.x)
    assert rel2(fem.normalise_pressure(N, host(x)), xo) <= 1e-8
    x = dev(xl)
    info = s.fgmres_solve(dev(b), x, rtol=0.0, restart=40, max_iters=36)
    assert info["iterations"] == 36 and info["restarts"] == 0
    assert info["status_name"] == "VKMG_ERR_NOT_CONVERGED"
    xh = host(x)
    r0 = np.linalg.norm(b - A @ xl)
    assert np.linalg.norm(b - A @ xh) <= 1e-12 * r0
    assert rel2(fem.normalise_pressure(N, xh), xo) <= 1e-8


def test_fgmres_edge_cases():
    N, levels = 16, 3
    s = solver(N, levels)
    g = grid_sizes(N)
    A, b, xl, _ = _manufactured_system(N)
    # zero right-hand side and zero guess: nothing to do
    z = dev(np.zeros(g.n))
    info = s.fgmres_solve(dev(np.zeros(g.n)), z)
    assert info["iterations"] == 0 and info["status_name"] == "VKMG_OK"
    # iteration cap
    x = dev(xl)
    info = s.fgmres_solve(dev(b), x, rtol=1e-14, max_iters=2)
    assert info["iterations"] == 2 and info["status_name"] == "VKMG_ERR_NOT_CONVERGED"
    # non-finite data is reported, not iterated on
    bn = b.copy()
    bn[5] = np.nan
    info = s.fgmres_solve(dev(bn), dev(xl))
    assert info["status_name"] == "VKMG_ERR_NONFINITE"
    # restart from the returned iterate (the iterate is the whole state)
    x = dev(xl)
    s.fgmres_solve(dev(b), x, rtol=1e-14, max_iters=3)
    info2 = s.fgmres_solve(dev(b), x, rtol=1e-6, max_iters=100)
    assert info2["status_name"] == "VKMG_OK"
    with pytest.raises(ValueError):
        s.vcycle(dev(np.zeros(g.n - 1)))
    n0 = s.level_layout(0)["n"]
    with pytest.raises(vk.VkmgError):  # level 0 is solved exactly, not relaxed
        s.vanka_sweep(0, dev(np.zeros(n0)), dev(np.zeros(n0)))


# ---------------------------------------------------------------- FP32 multigrid

@pytest.mark.parametrize("N,levels", [(16, 3), (40, 3)])
def test_fp32_multigrid_steps(N, levels):
    note(f"fp32 N={N}")
    s = solver(N, levels, "fp32")
    H = hierarchy(N, levels)
    lev = H.levels[-1]
    x, b = dirichlet_consistent_pair(N, 7, 8)
    xg = dev(x, torch.float32)
    s.vanka_sweep(levels - 1, xg, dev(b, torch.float32))
    xo = lev.smoother.sweep(x.astype(np.float32).astype(np.float64),
                            b.astype(np.float32).astype(np.float64))
    assert rel(host(xg), xo) < 1e-5
    r = uniform_vector(lev.n, 9)
    r[velocity_dirichlet_mask(N)] = 0
    z = host(s.vcycle(dev(r)))
    assert rel(z, H.vcycle(r)) < 1e-4


def test_fp32_multigrid_fgmres_reaches_fp64_tolerance():
    N, levels = 32, 4
    s32 = solver(N, levels, "fp32")
    H = hierarchy(N, levels)
    A, b, xl, _ = _manufactured_system(N)
    x = dev(xl)
    info = s32.fgmres_solve(dev(b), x, rtol=1e-8, restart=30, max_iters=200)
    assert info["status_name"] == "VKMG_OK" and info["true_rel_res"] <= 1e-8
    ro = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8)
    assert info["iterations"] <= ro.iterations + 3
    # both meet 1e-8 in the relative residual; the solutions agree to the
    # conditioning of the system times that tolerance
    xa = fem.normalise_pressure(N, host(x))
    xo = fem.normalise_pressure(N, ro.x)
    note(f"fp32-MG vs fp64 oracle rel err per field {rel2(xa, xo):.3e}")
    assert rel2(xa, xo) <= 1e-5


def test_kernel_timing_counts_launches():
    s = solver(16, 3)
    g = grid_sizes(16)
    s.set_timing(1 << vk.KERNEL_VANKA)
    s.vcycle(dev(np.zeros(g.n)))
    n, ms = s.kernel_timing(vk.KERNEL_VANKA)
    s.set_timing(0)
    # 2 relaxed levels x (2 + 2) sweeps; each sweep is one or two launches
    # (interior and boundary tiles) bracketed by one event pair
    assert n == 8 and ms > 0.0
