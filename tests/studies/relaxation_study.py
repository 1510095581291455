"""Iteration study of the relaxation schemes with the CPU oracle.

    python tests/studies/relaxation_study.py > tests/studies/relaxation_study.txt

Runs only the oracle (plain NumPy/SciPy FP64).  Two questions:

1. Vanka against Braess-Sarazin.  FGMRES(30) iterations to rtol 1e-8 from
   x0 = 0 for the Gaussian-random-field body force (length 0.1, unit
   variance, seed 5, homogeneous Dirichlet data; the benchmark workload on
   smaller meshes, coarsest mesh 8 x 8), under V(1,1) (the paper's cycle)
   and V(2,2), for additive Vanka with the partition-of-unity weights
   W_i = omega diag(1/m_j) (several omega) and with a plain scalar weight
   W_i = omega I (the other reading of the paper's unspecified weight
   matrix), and for inexact Braess-Sarazin (t = 1, omega_BS = 1; two
   Jacobi sweeps of weight 1 on the Schur complement, the library's
   default, or one sweep of weight 0.8 or 0.6).

2. Coarse operators for a per-element viscosity (log nu ~ U[-1, 1], seed
   7): rediscretisation with the mean of the four children against the
   Galerkin product P^T A P; FGMRES iterations and the asymptotic V(2,2)
   contraction factor (power iteration on the error propagator).
"""

from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fem, fgmres, multigrid  # noqa: E402
from stokes_inputs import (gaussian_random_field, grid_sizes, log_viscosity_field,  # noqa: E402
                           velocity_dirichlet_mask)


def levels_for(N):
    return int(np.log2(N // 8)) + 1


def solve_count(H, b, max_iters=80):
    n = b.size
    res = fgmres.fgmres(H.A, b, np.zeros(n), H.vcycle, rtol=1e-8, restart=30,
                        max_iters=max_iters)
    return res.iterations if res.converged else None


def contraction(H, N, steps=12, seed=3):
    A = H.A
    off_p = grid_sizes(N).off_p
    e = np.random.default_rng(seed).standard_normal(A.shape[0])
    e[velocity_dirichlet_mask(N)] = 0.0
    rho = 0.0
    for _ in range(steps):
        e2 = e - H.vcycle(A @ e)
        e2[off_p:] -= e2[off_p:].mean()
        rho = np.linalg.norm(e2) / np.linalg.norm(e)
        e = e2 / np.linalg.norm(e2)
    return rho


def fmt(v):
    return "div/>80" if v is None else str(v)


def study_relaxation(sizes):
    print("## Vanka vs Braess-Sarazin: FGMRES(30) iterations to 1e-8 (GRF force, seed 5)\n")
    rows = [("Vanka, W = omega diag(1/m_j), omega = 0.5", "vanka", 0.5, "pou"),
            ("Vanka, W = omega diag(1/m_j), omega = 0.75", "vanka", 0.75, "pou"),
            ("Vanka, W = omega diag(1/m_j), omega = 1.0", "vanka", 1.0, "pou"),
            ("Vanka, W = omega I, omega = 0.1", "vanka", 0.1, "scalar"),
            ("Vanka, W = omega I, omega = 0.15", "vanka", 0.15, "scalar"),
            ("Vanka, W = omega I, omega = 0.2", "vanka", 0.2, "scalar"),
            ("Vanka, W = omega I, omega = 0.3", "vanka", 0.3, "scalar"),
            ("Braess-Sarazin (t = 1, omega_BS = 1, Jacobi 2 x weight 1)", "bs", None,
             dict(jacobi_sweeps=2, jacobi_weight=1.0)),
            ("Braess-Sarazin (t = 1, omega_BS = 1, Jacobi 1 x weight 0.8)", "bs", None,
             dict(jacobi_sweeps=1, jacobi_weight=0.8)),
            ("Braess-Sarazin (t = 1, omega_BS = 1, Jacobi 1 x weight 0.6)", "bs", None,
             dict(jacobi_sweeps=1, jacobi_weight=0.6))]
    header = "| Relaxation | " + " | ".join(
        f"{N}^2 V({c},{c})" for N in sizes for c in (1, 2)) + " |"
    print(header)
    print("|" + "---|" * (1 + 2 * len(sizes)))
    data = {}
    for N in sizes:
        f = gaussian_random_field(N, 5, length=0.1)
        _, b, _, _ = fem.stokes_system(N, 1.0, f_nodal=f)
        L = levels_for(N)
        for c in (1, 2):
            for name, relax, omega, mode in rows:
                t0 = time.perf_counter()
                if relax == "bs":
                    H = multigrid.Hierarchy(N, L, nu_pre=c, nu_post=c, relaxation="bs", bs=mode)
                else:
                    H = multigrid.Hierarchy(N, L, omega=omega, nu_pre=c, nu_post=c)
                    if mode == "scalar":
                        for lev in H.levels[1:]:
                            w = np.full(lev.n, omega)
                            w[lev.dmask] = 0.0
                            lev.smoother.w = w
                data[(name, N, c)] = solve_count(H, b)
                print(f"[{N} V({c},{c}) {name}: {fmt(data[(name, N, c)])}, "
                      f"{time.perf_counter() - t0:.1f} s]", file=sys.stderr, flush=True)
    for name, *_ in rows:
        print(f"| {name} | " + " | ".join(fmt(data[(name, N, c)]) for N in sizes
                                          for c in (1, 2)) + " |")
    print()


def study_coarse_viscosity(sizes):
    print("## Per-element viscosity (log nu ~ U[-1,1], seed 7): coarse operators, "
          "V(2,2) Vanka omega = 0.5\n")
    print("| N | levels | coarse operator | FGMRES iterations | V-cycle contraction |")
    print("|---|---|---|---|---|")
    for N in sizes:
        L = levels_for(N)
        nu = np.exp(log_viscosity_field(N, 7))
        f = gaussian_random_field(N, 5, length=0.1)
        _, b, _, _ = fem.stokes_system(N, nu, f_nodal=f)
        for mode in ("rediscretise", "galerkin"):
            t0 = time.perf_counter()
            H = multigrid.Hierarchy(N, L, nu=nu, coarse_operator=mode)
            it = solve_count(H, b)
            rho = contraction(H, N)
            print(f"| {N} | {L} | {mode} | {fmt(it)} | {rho:.3f} |", flush=True)
            print(f"[{N} {mode}: {time.perf_counter() - t0:.1f} s]", file=sys.stderr, flush=True)
    print()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[64, 128, 256])
    ap.add_argument("--viscosity-sizes", type=int, nargs="+", default=[32, 64, 128])
    ap.add_argument("--skip-relaxation", action="store_true")
    ap.add_argument("--skip-viscosity", action="store_true")
    a = ap.parse_args()
    if not a.skip_relaxation:
        study_relaxation(a.sizes)
    if not a.skip_viscosity:
        study_coarse_viscosity(a.viscosity_sizes)


if __name__ == "__main__":
    main()
