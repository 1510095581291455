"""Write the oracle's reference values for the 1024 x 1024, 8-level workload.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``stokes_inputs/``).  The workload is the benchmark's: Q2-Q1 Stokes on the
unit square with 1024 x 1024 elements, nu = 1, homogeneous Dirichlet velocity,
body force a Gaussian random field (length 0.1, unit variance, seed 5) loaded
as b_u = M_Q2 f, x0 = 0; multigrid of the paper's Algorithm 1 with 8 levels,
V(2,2) additive Vanka (omega = 0.5, weights omega/m_j), coarsest 8 x 8 solved
exactly; FGMRES(30) to rtol 1e-8 ("Overall solver performance").  The Vanka
patch inverses are class-shared (one representative per boundary-distance
class, the paper's "tuned" Vanka); the oracle's CPU tests show that this
equals extracting every patch on meshes up to 64 x 64.

Output: ``c3_oracle_1024.json`` beside this script, holding
  * the FGMRES iteration count at rtol 1e-8 and the true relative residual;
  * the solution after that many iterations (pressure reduced to zero
    mass-weighted mean) at sampled DoFs, with the whole vector's maximum
    magnitude per field (u_x, u_y, p);
  * the output of one V-cycle z = M r for r ~ U[-1,1] (seed 170, zero on the
    Dirichlet DoFs) at the same DoFs, with its maximum magnitude per field.

The sampled DoFs are the corners, edges and the first rows in from the
boundary, seams of 14- and 16-element tiles, and random DoFs (seed 171),
about 6000 per vector.

Run: ``python tests/golden/make_c3_oracle.py`` (about 15 minutes and 30 GB of
host memory on 8 cores).
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fem, fgmres, multigrid  # noqa: E402
from stokes_inputs import (gaussian_random_field, grid_sizes, uniform_vector,  # noqa: E402
                           velocity_dirichlet_mask)

N, LEVELS = 1024, 8
FORCE_SEED, VCYCLE_SEED, SAMPLE_SEED = 5, 170, 171
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle_1024.json")


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def sample_dofs(N: int, seed: int, per_field_random: int = 1500) -> np.ndarray:
    g = grid_sizes(N)
    s2, s1 = g.q2_side, g.q1_side
    near2 = sorted({0, 1, 2, 3, 4, 5, 6, 7} | {s2 - 1 - k for k in range(8)}
                   | {2 * 14 * t + d for t in (1, 2, 36) for d in (-1, 0, 1)}
                   | {2 * 16 * t + d for t in (1, 2, 32) for d in (-1, 0, 1)})
    near1 = sorted({0, 1, 2, 3, 4, s1 - 5, s1 - 4, s1 - 3, s1 - 2, s1 - 1}
                   | {14 * t + d for t in (1, 2, 36) for d in (-1, 0, 1)}
                   | {16 * t + d for t in (1, 2, 32) for d in (-1, 0, 1)})
    near2 = [v for v in near2 if 0 <= v < s2]
    near1 = [v for v in near1 if 0 <= v < s1]
    dofs = set()
    # every (i, j) pair of the structured rows/columns near the boundary and
    # tile seams would be too many: take each structured row against a
    # spread of columns
    for k, j in enumerate(near2):
        for i in near2[k % 3::3]:
            dofs.add(g.off_ux + j * s2 + i)
            dofs.add(g.off_uy + i * s2 + j)
    for k, J in enumerate(near1):
        for I in near1[k % 2::2]:
            dofs.add(g.off_p + J * s1 + I)
    rng = np.random.default_rng(seed)
    dofs.update(int(v) for v in rng.integers(g.off_ux, g.off_uy, per_field_random))
    dofs.update(int(v) for v in rng.integers(g.off_uy, g.off_p, per_field_random))
    dofs.update(int(v) for v in rng.integers(g.off_p, g.n, per_field_random))
    return np.array(sorted(dofs), dtype=np.int64)


def field_max(N: int, v: np.ndarray):
    g = grid_sizes(N)
    return [float(np.abs(v[g.off_ux:g.off_uy]).max()), float(np.abs(v[g.off_uy:g.off_p]).max()),
            float(np.abs(v[g.off_p:]).max())]


def main():
    g = grid_sizes(N)
    dmask = velocity_dirichlet_mask(N)
    t0 = time.time()
    log(f"hierarchy N={N} levels={LEVELS} (assembly, class-shared patch inverses)")
    H = multigrid.Hierarchy(N, LEVELS)
    t_setup = time.time() - t0
    log(f"hierarchy done in {t_setup:.0f} s")
    A = H.A

    # the load of the random force with homogeneous Dirichlet data: with
    # g = 0 the elimination only sets the Dirichlet entries of b to 0
    f = gaussian_random_field(N, FORCE_SEED, length=0.1)
    b = fem.rhs_from_nodal_force(N, f)
    b[dmask] = 0.0

    dofs = sample_dofs(N, SAMPLE_SEED)
    log(f"{len(dofs)} sampled DoFs")

    log("one V-cycle")
    r = uniform_vector(g.n, VCYCLE_SEED)
    r[dmask] = 0.0
    t1 = time.time()
    z = H.vcycle(r)
    t_vc = time.time() - t1
    log(f"V-cycle {t_vc:.1f} s")

    log("FGMRES(30), rtol 1e-8, x0 = 0")
    calls = [0]

    def precond(v):
        calls[0] += 1
        log(f"  V-cycle {calls[0]}")
        return H.vcycle(v)

    t1 = time.time()
    res = fgmres.fgmres(A, b, np.zeros(g.n), precond, rtol=1e-8, restart=30, max_iters=500)
    t_solve = time.time() - t1
    log(f"FGMRES: {res.iterations} iterations, true rel res {res.true_rel_res:.3e}, {t_solve:.0f} s")
    x = fem.normalise_pressure(N, res.x)

    out = {
        "workload": ("Q2-Q1 Stokes, 1024x1024 elements, nu=1, homogeneous Dirichlet velocity, "
                     "GRF body force (length 0.1, unit variance, seed 5), b_u = M_Q2 f, x0 = 0; "
                     "8 levels, V(2,2) additive Vanka omega=0.5 (weights omega/m_j), class-shared "
                     "patch inverses, coarsest 8x8 exact (bordered); FGMRES(30), rtol 1e-8"),
        "written_by": "tests/golden/make_c3_oracle.py (CPU oracle only)",
        "N": N,
        "levels": LEVELS,
        "iterations": int(res.iterations),
        "restarts": int(res.restarts),
        "true_rel_res": float(res.true_rel_res),
        "est_history": [float(v) for v in res.est_history],
        "vcycle_input": {"kind": "uniform[-1,1], zero on Dirichlet DoFs", "seed": VCYCLE_SEED},
        "dofs": [int(d) for d in dofs],
        "solution": [float(v) for v in x[dofs]],
        "solution_field_max": field_max(N, x),
        "solution_field_norm": [float(np.linalg.norm(x[g.off_ux:g.off_uy])),
                                float(np.linalg.norm(x[g.off_uy:g.off_p])),
                                float(np.linalg.norm(x[g.off_p:]))],
        "vcycle": [float(v) for v in z[dofs]],
        "vcycle_field_max": field_max(N, z),
        "oracle_seconds": {"setup": t_setup, "vcycle": t_vc, "fgmres": t_solve},
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)
        fh.write("\n")
    log(f"wrote {OUT}")


if __name__ == "__main__":
    main()
