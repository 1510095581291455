"""Write the oracle's reference values for the 1024 x 1024, 8-level workload
with Braess-Sarazin relaxation.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``stokes_inputs/``).  The workload is the benchmark's Braess-Sarazin
comparison: Q2-Q1 Stokes on the unit square with 1024 x 1024 elements, nu = 1,
homogeneous Dirichlet velocity, body force a Gaussian random field (length
0.1, unit variance, seed 5), x0 = 0; multigrid of the paper's Algorithm 1 with
8 levels, V(2,2) inexact Braess-Sarazin relaxation (the paper's Algorithm 2
with t = 1, omega_BS = 1, two weighted-Jacobi sweeps of weight 1 on the Schur
system), coarsest 8 x 8 solved exactly; FGMRES(30) to rtol 1e-8.

Output: ``bs_oracle_1024.json`` beside this script, holding the FGMRES
iteration count at rtol 1e-8, the true relative residual, and the solution
after that many iterations (pressure reduced to zero mass-weighted mean) at
sampled DoFs, with the whole vector's maximum magnitude per field (u_x, u_y,
p).  The sampled DoFs are the corners, edges and first rows in from the
boundary, the seams of 14- and 16-element tiles, and random DoFs (seed 1023),
about 5000 per vector.

Run: ``python tests/golden/make_bs_oracle.py`` (several minutes and about
30 GB of host memory on 8 cores).
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
from stokes_inputs import gaussian_random_field, grid_sizes  # noqa: E402

N, LEVELS = 1024, 8
FORCE_SEED, SAMPLE_SEED = 5, 1023
BS = dict(t=1.0, omega_bs=1.0, jacobi_weight=1.0, jacobi_sweeps=2)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bs_oracle_1024.json")


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def sample_dofs(N: int, seed: int, per_field_random: int = 1200) -> np.ndarray:
    """Structured rows and columns (boundary, first rows in, tile seams of
    both tile sizes) crossed with a spread of each other, plus random DoFs."""
    g = grid_sizes(N)
    s2, s1 = g.q2_side, g.q1_side
    seams2 = {2 * 14 * t + d for t in (1, 2, N // 14) for d in (-1, 0, 1)}
    seams2 |= {2 * 16 * t + d for t in (1, 2, N // 16) for d in (-1, 0, 1)}
    seams1 = {14 * t + d for t in (1, 2, N // 14) for d in (-1, 0, 1)}
    seams1 |= {16 * t + d for t in (1, 2, N // 16) for d in (-1, 0, 1)}
    near2 = sorted(v for v in ({0, 1, 2, 3, 4, 5} | {s2 - 1 - k for k in range(6)} | seams2)
                   if 0 <= v < s2)
    near1 = sorted(v for v in ({0, 1, 2, 3, s1 - 4, s1 - 3, s1 - 2, s1 - 1} | seams1)
                   if 0 <= v < s1)
    dofs = set()
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
    t0 = time.time()
    log(f"hierarchy N={N} levels={LEVELS}, Braess-Sarazin relaxation {BS}")
    H = multigrid.Hierarchy(N, LEVELS, relaxation="bs", bs=BS,
                            progress=lambda m: log(f"  {m}"))
    log(f"hierarchy done in {time.time() - t0:.0f} s")
    dofs = sample_dofs(N, SAMPLE_SEED, per_field_random=1200)
    log(f"{len(dofs)} sampled DoFs")
    A, b, _, xl = fem.stokes_system(N, 1.0, f_nodal=gaussian_random_field(N, FORCE_SEED))
    t1 = time.time()
    res = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8, restart=30, max_iters=500)
    log(f"{res.iterations} iterations, true rel res {res.true_rel_res:.3e}, "
        f"{time.time() - t1:.0f} s")
    x = fem.normalise_pressure(N, res.x)
    out = {
        "workload": ("Q2-Q1 Stokes, 1024x1024 elements, nu=1, homogeneous Dirichlet velocity, "
                     "GRF body force (length 0.1, unit variance, seed 5), x0 = 0; 8 levels, "
                     "V(2,2) inexact Braess-Sarazin relaxation (t=1, omega_BS=1, two Jacobi "
                     "sweeps of weight 1), coarsest 8x8 exact (bordered); FGMRES(30), rtol 1e-8"),
        "written_by": "tests/golden/make_bs_oracle.py (CPU oracle only)",
        "N": N,
        "levels": LEVELS,
        "bs": BS,
        "iterations": int(res.iterations),
        "true_rel_res": float(res.true_rel_res),
        "dofs": [int(d) for d in dofs],
        "solution": [float(v) for v in x[dofs]],
        "solution_field_max": field_max(N, x),
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)
        fh.write("\n")
    log(f"wrote {OUT}")


if __name__ == "__main__":
    main()
