"""GPU parity of the per-element viscosity path (vkmg_setup_viscosity:
element-wise residual, one stored inverse per Vanka patch, averaged coarse
viscosities) against the oracle built with the same field.  Tolerances as
for the constant-viscosity path: operator 1e-13, one sweep 1e-12, V-cycle
1e-11, FGMRES iterations +-1 and the solution at equal iteration counts
1e-10, each per field (u_x, u_y, p against their own magnitudes).  Field:
log nu_e ~ U[-1, 1] (seeded)."""

import numpy as np
import pytest

from oracle import fem, fgmres, multigrid
from stokes_inputs import (dirichlet_consistent_pair, gaussian_random_field, grid_sizes,
                           log_viscosity_field, uniform_vector, velocity_dirichlet_mask)

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


def _nu(N, seed=7):
    return np.exp(log_viscosity_field(N, seed))


@pytest.mark.parametrize("N,levels", [(16, 3), (24, 3), (40, 3)])
def test_variable_viscosity_operator_and_sweeps(N, levels):
    note(f"varnu N={N}")
    nu = _nu(N)
    s = vk.VkmgSolver(N, levels, nu_elem=nu)
    H = multigrid.Hierarchy(N, levels, nu=nu)
    g = grid_sizes(N)
    x = uniform_vector(g.n, 11)
    b = uniform_vector(g.n, 12)
    assert rel(host(s.residual(dev(b), dev(x))), b - H.A @ x) < 1e-13
    assert rel(host(s.apply(dev(x))), H.A @ x) < 1e-13
    for l in range(1, levels):
        lev = H.levels[l]
        note(f"varnu N={N} level={l}")
        xl, bl = dirichlet_consistent_pair(lev.N, 30 + l, 40 + l)
        xg = dev(xl)
        s.vanka_sweep(l, xg, dev(bl))
        xo = lev.smoother.sweep(xl, bl)
        assert rel(host(xg), xo) < 1e-12
        s.relax(l, xg, dev(bl))
        assert rel(host(xg), lev.smoother.sweep(xo, bl)) < 1e-12
    r = uniform_vector(g.n, 13)
    r[velocity_dirichlet_mask(N)] = 0.0
    assert rel(host(s.vcycle(dev(r))), H.vcycle(r)) < 1e-11
    s.close()


def test_variable_viscosity_fp32_sweep():
    N, levels = 24, 3
    nu = _nu(N)
    s = vk.VkmgSolver(N, levels, nu_elem=nu, precision="fp32")
    H = multigrid.Hierarchy(N, levels, nu=nu)
    lev = H.levels[-1]
    xl, bl = dirichlet_consistent_pair(N, 50, 51)
    xg = dev(xl, torch.float32)
    s.vanka_sweep(levels - 1, xg, dev(bl, torch.float32))
    xo = lev.smoother.sweep(xl.astype(np.float32).astype(np.float64),
                            bl.astype(np.float32).astype(np.float64))
    assert rel(host(xg), xo) < 1e-5
    s.close()


@pytest.mark.parametrize("N,levels", [(16, 3), (32, 4)])
def test_variable_viscosity_fgmres(N, levels):
    note(f"varnu fgmres N={N}")
    nu = _nu(N)
    s = vk.VkmgSolver(N, levels, nu_elem=nu)
    H = multigrid.Hierarchy(N, levels, nu=nu)
    f = gaussian_random_field(N, 14, length=0.2)
    A, b, _, xl = fem.stokes_system(N, nu, f_nodal=f)
    ro = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8, restart=30, max_iters=200)
    bg = s.assemble_rhs(dev(f.ravel()))
    assert rel(host(bg), b) < 1e-13
    x = dev(xl)
    info = s.fgmres_solve(bg, x, rtol=1e-8, restart=30, max_iters=200)
    assert info["status_name"] == "VKMG_OK"
    assert abs(info["iterations"] - ro.iterations) <= 1
    k = ro.iterations
    x = dev(xl)
    info_k = s.fgmres_solve(bg, x, rtol=0.0, restart=30, max_iters=k)
    assert info_k["iterations"] == k
    ok = fgmres.fgmres(A, b, xl, H.vcycle, rtol=0.0, restart=30, fixed_iters=k)
    xa = fem.normalise_pressure(N, host(x))
    xo = fem.normalise_pressure(N, ok.x)
    assert rel2(xa, xo) <= 1e-10
    s.close()


def test_constant_field_matches_the_shared_inverse_path():
    """A constant field through the per-patch path equals the constant
    viscosity solver (stored inverses vs the symmetry-form apply)."""
    N, levels = 24, 3
    sv = vk.VkmgSolver(N, levels, nu_elem=np.full(N * N, 1.7))
    sc = vk.VkmgSolver(N, levels, nu=1.7)
    r = uniform_vector(grid_sizes(N).n, 60)
    r[velocity_dirichlet_mask(N)] = 0.0
    assert rel(host(sv.vcycle(dev(r))), host(sc.vcycle(dev(r)))) < 1e-11
    sv.close()
    sc.close()


def test_variable_viscosity_batched_equals_single_bitwise():
    N, levels, B = 24, 3, 2
    nu = _nu(N)
    sb = vk.VkmgSolver(N, levels, nu_elem=nu, batch=B)
    s1 = vk.VkmgSolver(N, levels, nu_elem=nu)
    n = s1.layout["n"]
    rs = [uniform_vector(n, 70 + k) for k in range(B)]
    zb = host(sb.vcycle(dev(np.concatenate(rs)))).reshape(B, n)
    for k in range(B):
        assert np.array_equal(zb[k], host(s1.vcycle(dev(rs[k]))))
    sb.close()
    s1.close()
