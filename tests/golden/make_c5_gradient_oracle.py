"""Write the oracle's gradients for the 256 x 256, 6-level per-element
viscosity workload.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``stokes_inputs/``).  Workload: Q2-Q1 Stokes on the unit square with
256 x 256 elements, per-element viscosity nu_e = exp(theta_e), theta ~
U[-1, 1] (seed 7), homogeneous Dirichlet velocity, body force f a Gaussian
random field (length 0.1, unit variance, seed 5); solution x_hat with zero
plain-mean pressure; loss L = |x_hat - x_t|^2 / 2 with x_t = 0.01 times a
Gaussian random field (length 0.1, seed 6) on the velocity and zero on the
pressure.  The gradients dL/df (per nodal force value) and dL/dnu_e come
from the forward and adjoint solves (A symmetric) of the oracle's
multigrid-preconditioned FGMRES (Algorithm 1 with 6 levels, V(2,2) additive
Vanka with one inverse per patch, omega = 0.5; FGMRES(30)) to rtol 1e-10,
mapped back by the adjoint formulas (``oracle.adjoint``).

Output: ``c5_gradient_oracle_256.json`` beside this script, holding the loss,
both FGMRES iteration counts, the largest magnitude of each gradient, and
each gradient at sampled entries: the force gradient at nodes on and next to
the boundary, on the seams of 14- and 16-element tiles and at random, in
both components; the viscosity gradient at elements along the boundary, the
tile seams and at random.

Run: ``python tests/golden/make_c5_gradient_oracle.py`` (a few minutes on 8
cores).
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint  # noqa: E402
from stokes_inputs import gaussian_random_field, grid_sizes, log_viscosity_field  # noqa: E402

N, LEVELS = 256, 6
FORCE_SEED, TARGET_SEED, NU_SEED, SAMPLE_SEED = 5, 6, 7, 257
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_gradient_oracle_256.json")


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def sample_force_entries(N: int, seed: int, n_random: int = 1500) -> np.ndarray:
    """Indices into the force array raveled as (2, (2N+1)^2): boundary and
    first rows in, tile seams, crossed with a spread of each other, plus
    random nodes, both components."""
    s2 = 2 * N + 1
    seams = {2 * 14 * t + d for t in (1, 2, N // 14) for d in (-1, 0, 1)}
    seams |= {2 * 16 * t + d for t in (1, 2, N // 16) for d in (-1, 0, 1)}
    near = sorted(v for v in ({0, 1, 2, 3, 4, 5} | {s2 - 1 - k for k in range(6)} | seams)
                  if 0 <= v < s2)
    idx = set()
    for k, j in enumerate(near):
        for i in near[k % 3::3]:
            idx.add(j * s2 + i)
            idx.add(s2 * s2 + i * s2 + j)
    rng = np.random.default_rng(seed)
    idx.update(int(v) for v in rng.integers(0, 2 * s2 * s2, n_random))
    return np.array(sorted(idx), dtype=np.int64)


def sample_elements(N: int, seed: int, n_random: int = 1500) -> np.ndarray:
    """Element indices ey*N + ex along the boundary, the tile seams and at
    random."""
    seams = {14 * t + d for t in (1, 2, N // 14) for d in (-1, 0)}
    seams |= {16 * t + d for t in (1, 2, N // 16) for d in (-1, 0)}
    near = sorted(v for v in ({0, 1, 2, N - 3, N - 2, N - 1} | seams) if 0 <= v < N)
    idx = set()
    for k, ey in enumerate(near):
        for ex in near[k % 2::2]:
            idx.add(ey * N + ex)
    rng = np.random.default_rng(seed + 1)
    idx.update(int(v) for v in rng.integers(0, N * N, n_random))
    return np.array(sorted(idx), dtype=np.int64)


def main():
    theta = log_viscosity_field(N, NU_SEED)
    nu = np.exp(theta)
    f = gaussian_random_field(N, FORCE_SEED, length=0.1)
    n = grid_sizes(N).n
    xt = np.zeros(n)
    xt[:2 * (2 * N + 1) ** 2] = 0.01 * gaussian_random_field(N, TARGET_SEED, length=0.1).ravel()
    t0 = time.time()
    log(f"forward and adjoint solves N={N} levels={LEVELS} (per-element viscosity), rtol 1e-10")
    x_hat, g_f, g_nu, fw, aw = adjoint.iterative_gradients(
        N, LEVELS, f, lambda xh: xh - xt, nu, rtol=1e-10, max_iters=300)
    log(f"forward {fw.iterations} iterations (true rel res {fw.true_rel_res:.2e}), adjoint "
        f"{aw.iterations} ({aw.true_rel_res:.2e}), {time.time() - t0:.0f} s")
    loss = 0.5 * float(np.sum((x_hat - xt) ** 2))
    gf = g_f.ravel()
    fi = sample_force_entries(N, SAMPLE_SEED)
    ei = sample_elements(N, SAMPLE_SEED)
    log(f"{len(fi)} force entries, {len(ei)} elements sampled; loss {loss:.6e}")
    out = {
        "workload": ("Q2-Q1 Stokes, 256x256 elements, per-element viscosity exp(U[-1,1]) seed 7, "
                     "homogeneous Dirichlet velocity, GRF body force (length 0.1, seed 5); "
                     "x_hat with zero plain-mean pressure; L = |x_hat - x_t|^2/2, x_t = 0.01 "
                     "GRF (length 0.1, seed 6) on the velocity; forward and adjoint solves by "
                     "FGMRES(30) with the 6-level V(2,2) Vanka cycle (one inverse per patch) "
                     "to rtol 1e-10"),
        "written_by": "tests/golden/make_c5_gradient_oracle.py (CPU oracle only)",
        "N": N,
        "levels": LEVELS,
        "loss": loss,
        "forward_iterations": int(fw.iterations),
        "adjoint_iterations": int(aw.iterations),
        "force_gradient_max": float(np.abs(gf).max()),
        "viscosity_gradient_max": float(np.abs(g_nu).max()),
        "force_entries": [int(i) for i in fi],
        "force_gradient": [float(v) for v in gf[fi]],
        "elements": [int(i) for i in ei],
        "viscosity_gradient": [float(v) for v in g_nu[ei]],
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)
        fh.write("\n")
    log(f"wrote {OUT}")


if __name__ == "__main__":
    main()
