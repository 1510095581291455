"""GPU checks of the workloads at their stated sizes.

C2 (256 x 256, 6 levels, trigonometric manufactured solution, x0 = Dirichlet
lifting): FGMRES(30) iteration count within one of the oracle's at rtol
1e-8, and after exactly the oracle's count the solution (pressure reduced
to zero mass-weighted mean) within 1e-10 per field, in FP64 multigrid; the
FP32-multigrid solve reaches the FP64 tolerance within one iteration of it.
The benchmark's standalone finest-level sweeps at this size (the update
given a seeded uniform[-1, 1] residual, and residual + update given x and
b) against the oracle's one-DoF-at-a-time sweep at sampled DoFs (corners,
edges, tile seams, random), 1e-12 of each field's maximum.

C4 (512 x 512, 7 levels, 32 right-hand sides: Gaussian random forces seeds
1000 + k under the watertight lid): one batched solve against 32 single
solves of the same systems: iteration counts equal and solutions bitwise
equal (batched launches do the arithmetic of single ones, and every batch
entry is reduced over the same partial sums as a single right-hand side);
and, in FP64 multigrid, the batch entries 0 and 31 against the oracle's
solves of those systems (tests/golden/c4_oracle_512.json, written by
tests/golden/make_c4_oracle.py): iteration counts within one at rtol 1e-8,
and after exactly the oracle's count the solutions within 1e-10 of each
field's maximum at the sampled DoFs and the true relative residuals equal
to the oracle's to 1e-3 relative; with the V-cycle in FP32 (the precision
this workload names) the same iteration bound, then the true residuals at
the tolerance and the solutions within 1e-8 per field.

C5 forward solve (256 x 256, 6 levels, log nu ~ U[-1, 1] seed 7, Gaussian
random force seed 5, one inverse per patch): against the oracle's solve
(tests/golden/c5_oracle_256.json, written by tests/golden/make_c5_oracle.py):
iteration count within one at rtol 1e-8, and after exactly the oracle's
count the solution within 1e-10 of each field's maximum at the sampled DoFs
and the true relative residual equal to the oracle's to 1e-3 relative
(with the V-cycle in FP32: residual at the tolerance, solution within 1e-8).

C5 gradients (the same viscosity and force, L = |x - x_t|^2 / 2 with
x_t = 0.01 GRF seed 6 on the velocity):
the autograd gradients with respect to the log-viscosity and the force
against central differences of the GPU solve on 20 seeded directions
(seed 8), 1e-6 relative (solves at rtol 1e-10: with this viscosity field
the adjoint system's FP64 rounding floor at 256 x 256 is a relative
residual of about 1.5e-11, so 1e-12 is out of reach); and the same
gradients against the oracle's adjoint gradients
(tests/golden/c5_gradient_oracle_256.json, written by
tests/golden/make_c5_gradient_oracle.py): loss to 1e-8 relative, each
gradient within 1e-6 of its largest magnitude at sampled entries.
"""

import numpy as np
import pytest

from oracle import fem, fgmres, multigrid, vanka
from stokes_inputs import (dirichlet_consistent_pair, gaussian_random_field, grid_sizes,
                           lid_boundary_values, log_viscosity_field, manufactured_boundary_values,
                           manufactured_nodal_force, uniform_vector, velocity_dirichlet_mask)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2401_06277_amd as vk  # noqa: E402
from fieldwise import rel  # noqa: E402
from paper_2401_06277_amd.autograd import stokes_solve  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def test_c2_manufactured_solve_matches_oracle():
    N, levels = 256, 6
    note(f"[C2] oracle solve N={N} levels={levels}")
    f = manufactured_nodal_force(N, "trig")
    g = manufactured_boundary_values(N, "trig")
    A, b, _, xl = fem.stokes_system(N, 1.0, f_nodal=f, g_nodal=g)
    H = multigrid.Hierarchy(N, levels)
    ro = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8)
    k = ro.iterations
    rk = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8, fixed_iters=k)
    xo = fem.normalise_pressure(N, rk.x)
    for prec in ("fp64", "fp32"):
        note(f"[C2] GPU {prec}")
        with vk.VkmgSolver(N, levels, precision=prec) as s:
            bd = s.assemble_rhs(dev(f.ravel()), dev(g.ravel()))
            assert rel(host(bd), b) <= 1e-13
            x = s.dirichlet_lift(bd)
            x0 = x.clone()
            info = s.fgmres_solve(bd, x, rtol=1e-8)
            note(f"[C2] {prec}: {info}; oracle {k} iterations")
            assert info["status_name"] == "VKMG_OK"
            assert abs(info["iterations"] - k) <= 1
            assert info["true_rel_res"] <= 1e-8
            if prec == "fp64":
                x = x0.clone()
                info_k = s.fgmres_solve(bd, x, rtol=0.0, max_iters=k)
                assert info_k["iterations"] == k
                xg = fem.normalise_pressure(N, host(x))
                err = rel(xg, xo)
                note(f"[C2] solution after {k} steps vs oracle: {err:.2e} (worst field)")
                assert err <= 1e-10



def _c2_sample_dofs(N, seed, n_random=400):
    """Corners, edges, one and two elements in, the seams of 14- and
    16-element tiles, and random DoFs, in all three fields."""
    g = grid_sizes(N)
    s2, s1 = g.q2_side, g.q1_side
    near = sorted({0, 1, 2, 3, 4, 5} | {s2 - 1 - k for k in range(6)}
                  | {2 * 14 - 1, 2 * 14, 2 * 14 + 1, 2 * 16, 2 * 16 + 1, s2 // 2})
    near1 = sorted({0, 1, 2, 3, s1 - 4, s1 - 3, s1 - 2, s1 - 1, 13, 14, 15, 16, 17, s1 // 2})
    dofs = []
    for i, qi in enumerate(near):
        qj = near[(3 * i + 1) % len(near)]
        dofs += [g.off_ux + qj * s2 + qi, g.off_uy + qi * s2 + qj]
    for k, I in enumerate(near1):
        dofs.append(g.off_p + near1[(5 * k + 2) % len(near1)] * s1 + I)
    rng = np.random.default_rng(seed)
    dofs += list(rng.choice(g.n, n_random, replace=False))
    return np.array(sorted(set(int(d) for d in dofs)))


def _fieldwise_close(N, got, want, dofs, tol, what):
    g = grid_sizes(N)
    field = np.searchsorted([g.off_uy, g.off_p], dofs, side="right")
    worst = []
    for f in range(3):
        sel = field == f
        assert sel.sum() > 5, (what, f)
        worst.append(float(np.abs(got[sel] - want[sel]).max() / max(np.abs(want[sel]).max(), 1e-300)))
    note(f"{what}: per-field max error {['%.2e' % e for e in worst]} at {len(dofs)} sampled DoFs")
    assert max(worst) <= tol, (what, worst)


def test_c2_standalone_sweeps_match_oracle():
    N, levels = 256, 6
    top = levels - 1
    g = grid_sizes(N)
    dofs = _c2_sample_dofs(N, 21)
    note(f"[C2 sweeps] N={N} levels={levels}: {len(dofs)} sampled DoFs")
    rin = uniform_vector(g.n, 2)
    rin[velocity_dirichlet_mask(N)] = 0.0
    xin, bin_ = dirichlet_consistent_pair(N, 3, 4)
    with vk.VkmgSolver(N, levels) as s:
        x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        s.vanka_update(top, x, dev(rin))
        got = host(x)[dofs]
        # x = 0: the sweep's residual is the given vector itself
        want = vanka.sampled_sweep_update(N, np.zeros(g.n), rin, dofs)
        _fieldwise_close(N, got, want, dofs, 1e-12, "[C2] update given r")
        x = dev(xin.copy())
        s.vanka_sweep(top, x, dev(bin_))
        got = host(x)[dofs] - xin[dofs]
        want = vanka.sampled_sweep_update(N, xin, bin_, dofs)
        _fieldwise_close(N, got, want, dofs, 1e-12, "[C2] residual + update given x, b")

def test_c4_batched_32_equals_single_solves():
    N, levels, B = 512, 7, 32
    note(f"[C4] N={N} levels={levels} batch={B}")
    fs = np.concatenate([gaussian_random_field(N, 1000 + k).ravel() for k in range(B)])
    g = lid_boundary_values(N).ravel()
    nq2 = (2 * N + 1) ** 2
    with vk.VkmgSolver(N, levels, precision="fp32", batch=B) as s:
        n = s.layout["n"]
        b = s.assemble_rhs(dev(fs), dev(np.tile(g, B)))
        x = s.dirichlet_lift(b)
        infos = s.fgmres_solve(b, x, rtol=1e-8)
        xb = host(x).reshape(B, n)
    with vk.VkmgSolver(N, levels, precision="fp32") as s1:
        worst = 0.0
        for k in range(B):
            bk = s1.assemble_rhs(dev(fs[2 * nq2 * k:2 * nq2 * (k + 1)]), dev(g))
            xk = s1.dirichlet_lift(bk)
            info = s1.fgmres_solve(bk, xk, rtol=1e-8)
            assert infos[k]["status_name"] == "VKMG_OK" and info["status_name"] == "VKMG_OK"
            assert infos[k]["iterations"] == info["iterations"], (k, infos[k], info)
            xs = host(xk)
            e = rel(xb[k], xs)
            worst = max(worst, e)
            assert np.array_equal(xb[k], xs), (k, e)
    note(f"[C4] {B} systems: iterations {[i['iterations'] for i in infos]}, "
         f"worst batched-vs-single difference {worst:.2e}")


def test_c4_batched_fp64_matches_oracle_golden():
    import json
    import os
    N, levels, B = 512, 7, 32
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_oracle_512.json")
    with open(path) as fh:
        d = json.load(fh)
    assert d["N"] == N and d["levels"] == levels
    note(f"[C4 golden] N={N} levels={levels} batch={B} fp64")
    fs = np.concatenate([gaussian_random_field(N, 1000 + k).ravel() for k in range(B)])
    g = lid_boundary_values(N).ravel()
    gs = grid_sizes(N)
    dofs = np.array(d["dofs"])
    field = np.searchsorted([gs.off_uy, gs.off_p], dofs, side="right")
    with vk.VkmgSolver(N, levels, precision="fp64", batch=B) as s:
        n = s.layout["n"]
        b = s.assemble_rhs(dev(fs), dev(np.tile(g, B)))
        x0 = s.dirichlet_lift(b)
        x = x0.clone()
        infos = s.fgmres_solve(b, x, rtol=1e-8)
        for k, ref in d["rhs"].items():
            k = int(k)
            note(f"[C4 golden] k={k}: GPU {infos[k]['iterations']} iterations, "
                 f"oracle {ref['iterations']}")
            assert infos[k]["status_name"] == "VKMG_OK"
            assert abs(infos[k]["iterations"] - ref["iterations"]) <= 1
        for m in sorted({ref["iterations"] for ref in d["rhs"].values()}):
            x = x0.clone()
            infos_m = s.fgmres_solve(b, x, rtol=0.0, max_iters=m)
            xb = host(x).reshape(B, n)
            for k, ref in d["rhs"].items():
                if ref["iterations"] != m:
                    continue
                k = int(k)
                assert infos_m[k]["iterations"] == m
                assert abs(infos_m[k]["true_rel_res"] - ref["true_rel_res"]) <= 1e-3 * ref["true_rel_res"]
                xn = fem.normalise_pressure(N, xb[k])
                want = np.array(ref["solution"])
                worst = []
                for f in range(3):
                    sel = field == f
                    assert sel.sum() > 1000
                    worst.append(np.abs(xn[dofs][sel] - want[sel]).max() / ref["solution_field_max"][f])
                note(f"[C4 golden] k={k} after {m} steps: per-field max error "
                     f"{['%.2e' % e for e in worst]}")
                assert max(worst) <= 1e-10, (k, worst)



def test_c4_batched_fp32_multigrid_matches_oracle_golden():
    """The 512 x 512 batch of 32 right-hand sides with the V-cycle in FP32
    (FGMRES, the Arnoldi process and the coarse solve in FP64) against the
    oracle's FP64 solves of entries 0 and 31 (tests/golden/make_c4_oracle.py):
    iteration counts within one at rtol 1e-8; after exactly the oracle's count
    the true relative residual at the tolerance and the solution within 1e-8
    of each field's maximum at the sampled DoFs.  As for the single FP32
    multigrid solve at 1024 x 1024, the FP32 cycle changes the Krylov path,
    so the iterates agree to their distance from the exact solution, which
    the tolerance sets, rather than to rounding (measured here: 2.3e-12 of
    each field's maximum, true residual 3.5e-9)."""
    import json
    import os
    N, levels, B = 512, 7, 32
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_oracle_512.json")
    with open(path) as fh:
        d = json.load(fh)
    assert d["N"] == N and d["levels"] == levels
    note(f"[C4 golden] N={N} levels={levels} batch={B} fp32 multigrid")
    fs = np.concatenate([gaussian_random_field(N, 1000 + k).ravel() for k in range(B)])
    g = lid_boundary_values(N).ravel()
    gs = grid_sizes(N)
    dofs = np.array(d["dofs"])
    with vk.VkmgSolver(N, levels, precision="fp32", batch=B) as s:
        n = s.layout["n"]
        b = s.assemble_rhs(dev(fs), dev(np.tile(g, B)))
        x0 = s.dirichlet_lift(b)
        x = x0.clone()
        infos = s.fgmres_solve(b, x, rtol=1e-8)
        for k, ref in d["rhs"].items():
            k = int(k)
            note(f"[C4 golden] k={k}: GPU (FP32 multigrid) {infos[k]['iterations']} iterations, "
                 f"oracle {ref['iterations']}")
            assert infos[k]["status_name"] == "VKMG_OK"
            assert abs(infos[k]["iterations"] - ref["iterations"]) <= 1
        for m in sorted({ref["iterations"] for ref in d["rhs"].values()}):
            x = x0.clone()
            infos_m = s.fgmres_solve(b, x, rtol=0.0, max_iters=m)
            xb = host(x).reshape(B, n)
            for k, ref in d["rhs"].items():
                if ref["iterations"] != m:
                    continue
                k = int(k)
                assert infos_m[k]["iterations"] == m
                assert infos_m[k]["true_rel_res"] <= 1e-8, (k, infos_m[k])
                xn = fem.normalise_pressure(N, xb[k])
                worst = _per_field(xn[dofs], np.array(ref["solution"]), dofs, gs,
                                   ref["solution_field_max"])
                note(f"[C4 golden] k={k} after {m} steps (FP32 multigrid): per-field max error "
                     f"{['%.2e' % e for e in worst]}, true rel res {infos_m[k]['true_rel_res']:.2e}")
                assert max(worst) <= 1e-8, (k, worst)

def _per_field(got, want, dofs, gs, field_max):
    field = np.searchsorted([gs.off_uy, gs.off_p], dofs, side="right")
    worst = []
    for f in range(3):
        sel = field == f
        assert sel.sum() > 1000
        worst.append(float(np.abs(got[sel] - want[sel]).max() / field_max[f]))
    return worst


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c5_forward_solve_matches_oracle_golden(precision):
    """With the V-cycle in FP32 (FGMRES in FP64) the bounds after the
    oracle's count are those of the FP32-multigrid solves: true residual at
    the tolerance, solution within 1e-8 per field."""
    import json
    import os
    N, levels = 256, 6
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_oracle_256.json")
    with open(path) as fh:
        d = json.load(fh)
    assert d["N"] == N and d["levels"] == levels
    note(f"[C5 golden] N={N} levels={levels} per-element viscosity, {precision} V-cycle")
    nu = np.exp(log_viscosity_field(N, 7))
    gs = grid_sizes(N)
    dofs = np.array(d["dofs"])
    with vk.VkmgSolver(N, levels, nu_elem=nu, precision=precision) as s:
        b = s.assemble_rhs(dev(gaussian_random_field(N, 5).ravel()))
        x = torch.zeros_like(b)
        info = s.fgmres_solve(b, x, rtol=1e-8)
        note(f"[C5 golden] GPU {info['iterations']} iterations, oracle {d['iterations']}")
        assert info["status_name"] == "VKMG_OK"
        assert abs(info["iterations"] - d["iterations"]) <= 1
        m = d["iterations"]
        x = torch.zeros_like(b)
        info_m = s.fgmres_solve(b, x, rtol=0.0, max_iters=m)
        assert info_m["iterations"] == m
        if precision == "fp64":
            assert abs(info_m["true_rel_res"] - d["true_rel_res"]) <= 1e-3 * d["true_rel_res"]
        else:
            assert info_m["true_rel_res"] <= 1e-8, info_m
        xn = fem.normalise_pressure(N, host(x))
        worst = _per_field(xn[dofs], np.array(d["solution"]), dofs, gs, d["solution_field_max"])
        note(f"[C5 golden] after {m} steps: per-field max error {['%.2e' % e for e in worst]}, "
             f"true rel res {info_m['true_rel_res']:.2e}")
        assert max(worst) <= (1e-10 if precision == "fp64" else 1e-8), worst


def test_c5_gradients_match_central_differences_at_256():
    N, levels = 256, 6
    note(f"[C5] N={N} levels={levels}")
    theta = log_viscosity_field(N, 7)
    f = gaussian_random_field(N, 5, length=0.1).ravel()
    n = grid_sizes(N).n
    xt = np.zeros(n)
    xt[:2 * (2 * N + 1) ** 2] = 0.01 * gaussian_random_field(N, 6, length=0.1).ravel()
    xt_d = dev(xt)

    # gradients by the adjoint (autograd over the solve) at theta
    nu = np.exp(theta)
    s = vk.VkmgSolver(N, levels, nu_elem=nu)
    fd = dev(f).requires_grad_(True)
    nud = dev(nu).requires_grad_(True)
    x = stokes_solve(fd, s, nu=nud, rtol=1e-10)
    (0.5 * torch.sum((x - xt_d) ** 2)).backward()
    g_theta, g_f = host(nud.grad) * nu, host(fd.grad)  # dL/dtheta = nu dL/dnu

    def loss(sv, force):
        with torch.no_grad():
            return float(0.5 * torch.sum((stokes_solve(dev(force), sv, rtol=1e-10) - xt_d) ** 2))

    rng = np.random.default_rng(8)
    eps = 1e-4
    worst_f = worst_t = 0.0
    for i in range(20):
        d = rng.standard_normal(f.shape)
        fdiff = (loss(s, f + eps * d) - loss(s, f - eps * d)) / (2 * eps)
        an = float(g_f @ d)
        worst_f = max(worst_f, abs(fdiff - an) / abs(an))
        assert abs(fdiff - an) <= 1e-6 * abs(an), ("force", i, fdiff, an)
    s.close()
    for i in range(20):
        d = rng.standard_normal(theta.shape)
        vals = []
        for sign in (1.0, -1.0):
            with vk.VkmgSolver(N, levels, nu_elem=np.exp(theta + sign * eps * d)) as sv:
                vals.append(loss(sv, f))
        fdiff = (vals[0] - vals[1]) / (2 * eps)
        an = float(g_theta @ d)
        worst_t = max(worst_t, abs(fdiff - an) / abs(an))
        assert abs(fdiff - an) <= 1e-6 * abs(an), ("log-viscosity", i, fdiff, an)
    note(f"[C5] worst relative FD mismatch: force {worst_f:.2e}, log-viscosity {worst_t:.2e}")


def test_c5_gradients_match_oracle_golden():
    """The autograd gradients at 256 x 256 (the C5 workload and loss of the
    central-difference test above) against the oracle's adjoint gradients
    (tests/golden/c5_gradient_oracle_256.json, written by
    tests/golden/make_c5_gradient_oracle.py from the oracle's forward and
    adjoint multigrid-FGMRES solves to rtol 1e-10): the loss to 1e-8
    relative, and each gradient at its sampled entries (nodes and elements on
    and next to the boundary, on tile seams and at random) within 1e-6 of its
    largest magnitude."""
    import json
    import os
    N, levels = 256, 6
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "c5_gradient_oracle_256.json")
    with open(path) as fh:
        d = json.load(fh)
    assert d["N"] == N and d["levels"] == levels
    note(f"[C5 gradient golden] N={N} levels={levels}")
    theta = log_viscosity_field(N, 7)
    nu = np.exp(theta)
    f = gaussian_random_field(N, 5, length=0.1).ravel()
    n = grid_sizes(N).n
    xt = np.zeros(n)
    xt[:2 * (2 * N + 1) ** 2] = 0.01 * gaussian_random_field(N, 6, length=0.1).ravel()
    with vk.VkmgSolver(N, levels, nu_elem=nu) as s:
        fd = dev(f).requires_grad_(True)
        nud = dev(nu).requires_grad_(True)
        x = stokes_solve(fd, s, nu=nud, rtol=1e-10)
        loss = 0.5 * torch.sum((x - dev(xt)) ** 2)
        loss.backward()
        g_f, g_nu = host(fd.grad), host(nud.grad)
    lv = float(loss.detach())
    e_loss = abs(lv - d["loss"]) / abs(d["loss"])
    fi, ei = np.array(d["force_entries"]), np.array(d["elements"])
    e_f = float(np.abs(g_f[fi] - np.array(d["force_gradient"])).max() / d["force_gradient_max"])
    e_nu = float(np.abs(g_nu[ei] - np.array(d["viscosity_gradient"])).max()
                 / d["viscosity_gradient_max"])
    note(f"[C5 gradient golden] loss {lv:.6e} vs {d['loss']:.6e} ({e_loss:.1e}); force gradient "
         f"{e_f:.2e} at {len(fi)} entries, viscosity gradient {e_nu:.2e} at {len(ei)} elements")
    assert e_loss <= 1e-8
    assert e_f <= 1e-6 and e_nu <= 1e-6, (e_f, e_nu)
