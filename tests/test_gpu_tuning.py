"""GPU tests of the launch-shape tuning (vkmg_tuning) and the fused sweep.

Every tuning choice (sweeps of a level fused into one launch, the parked
FP64 tile kernel, the coarse-grid correction inside the next residual,
boundary patches per wavefront) does the same arithmetic in the same order,
so V-cycles and FGMRES solves must be bitwise equal under any tuning; with
all fusion off the V-cycle is the three-launch form that the oracle tests
cover elementwise, so this also pins the fused sweep (every level from 16
elements per side, both precisions, batches, ragged tiles) to that form.
"""

import numpy as np
import pytest

from stokes_inputs import uniform_vector, velocity_dirichlet_mask

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2401_06277_amd as vk  # noqa: E402

NEVER = 2**31 - 1
PLAIN = dict(fused_sweep_max_n=0, park_min_n=NEVER, fused_prolong_max_n=0, boundary_per_wave=1)
ALL = dict(fused_sweep_max_n=NEVER, park_min_n=0, fused_prolong_max_n=NEVER, boundary_per_wave=8)
MIXED = dict(fused_sweep_max_n=32, park_min_n=64, fused_prolong_max_n=32, boundary_per_wave=2)


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


def _rhs(N, batch, seed):
    parts = []
    for k in range(batch):
        m = velocity_dirichlet_mask(N)  # over the whole vector
        r = uniform_vector(m.size, seed + k)
        r[m] = 0.0
        off_p = 2 * (2 * N + 1) ** 2
        r[off_p:] -= r[off_p:].mean()  # consistent with the constant-pressure null space
        parts.append(r)
    return torch.from_numpy(np.concatenate(parts)).cuda()


def _vcycles(s, r, tunings):
    outs = []
    for t in tunings:
        s.set_tuning(**t)
        z = torch.empty_like(r)
        s.vcycle(r, z)
        torch.cuda.synchronize()
        outs.append(z)
    return outs


@pytest.mark.parametrize("N,levels,prec,batch", [
    (64, 4, "fp64", 1), (64, 4, "fp32", 1), (48, 3, "fp64", 1), (48, 3, "fp32", 1),
    (32, 3, "fp64", 3), (256, 6, "fp64", 1), (256, 6, "fp32", 1)])
def test_vcycle_bitwise_under_every_tuning(N, levels, prec, batch):
    print(f"[tuning] vcycle N={N} levels={levels} {prec} batch={batch}", flush=True)
    with vk.VkmgSolver(N, levels, precision=prec, batch=batch) as s:
        r = _rhs(N, batch, 300)
        default = s.get_tuning()
        ref, *others = _vcycles(s, r, [PLAIN, ALL, MIXED, default])
        assert float(ref.abs().max()) > 0
        for z in others:
            assert torch.equal(z, ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fgmres_bitwise_under_tuning(prec):
    N, levels = 64, 4
    print(f"[tuning] fgmres N={N} {prec}", flush=True)
    with vk.VkmgSolver(N, levels, precision=prec) as s:
        b = _rhs(N, 1, 400)
        res = []
        for t in (PLAIN, ALL):
            s.set_tuning(**t)
            x = torch.zeros_like(b)
            info = s.fgmres_solve(b, x, rtol=1e-10)
            torch.cuda.synchronize()
            assert info["status_name"] == "VKMG_OK"
            res.append((info["iterations"], x))
        assert res[0][0] == res[1][0]
        assert torch.equal(res[0][1], res[1][1])


def test_set_tuning_rejects_invalid_values():
    with vk.VkmgSolver(32, 3) as s:
        before = s.get_tuning()
        for bad in (dict(boundary_per_wave=3), dict(park_min_n=-1), dict(fused_sweep_max_n=-5),
                    dict(fused_prolong_max_n=-1)):
            with pytest.raises(vk.VkmgError) as e:
                s.set_tuning(**bad)
            assert e.value.status_name == "VKMG_ERR_INVALID_ARG"
            assert s.get_tuning() == before


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotune_returns_valid_tuning_and_same_results(prec):
    N, levels = 128, 5
    print(f"[tuning] autotune N={N} {prec}", flush=True)
    with vk.VkmgSolver(N, levels, precision=prec) as s:
        r = _rhs(N, 1, 500)
        z0 = torch.empty_like(r)
        s.vcycle(r, z0)
        t = s.autotune(reps=3)
        print(f"  tuned: {t}", flush=True)
        assert t == s.get_tuning()
        assert t["boundary_per_wave"] in (0, 1, 2, 4, 8)
        assert min(t["fused_sweep_max_n"], t["park_min_n"], t["fused_prolong_max_n"]) >= 0
        z1 = torch.empty_like(r)
        s.vcycle(r, z1)
        torch.cuda.synchronize()
        assert torch.equal(z0, z1)
