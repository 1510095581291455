"""Benchmark: Vanka-multigrid-preconditioned FGMRES for Q2-Q1 Stokes on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--N 1024] [--levels 8]

Workload (default): 1024 x 1024 elements, 8 levels (coarsest 8 x 8), nu = 1,
homogeneous Dirichlet velocity, body force a seeded Gaussian random field
(length scale 0.1, unit variance, seed 5) on the Q2 nodes; V(2,2) additive
Vanka with omega = 0.5 inside FGMRES(30), rtol 1e-8.

A step is one complete FGMRES solve to rtol 1e-8 from the zero initial
guess (right-hand side resident in HBM), i.e. one pass of every step of the
hot path: residual, Vanka gather/apply/scatter, restriction, coarsest solve,
prolongation, V-cycle, Arnoldi/Givens and solution update.  The timed loop
runs K such solves with the plain FP64 path; ``value`` is the Vanka
patch-updates per second sustained over those solves (patch solves per
V-cycle x V-cycles / wall time).  A second timed loop of K solves with the
V-cycle in FP32 (FGMRES, Arnoldi and the coarse solve kept in FP64) is
reported under "fp32_mg".

Prints one JSON line.  The roofline object is for the dominant kernel, the
interior-tile kernel of the finest-level Vanka update (with the boundary-patch
kernel reported beside it), timed with HIP events on its launch stream in an
event-timed pass of the same K solves (kernel events bypass the captured
graphs); that pass also gives the per-class kernel time per solve
(kernel_ms_per_solve, krylov_share).  "c2_256" reports, at 256 x 256 with 6
levels, the standalone sweep rates (apply only given r, and residual +
update given x and b) and the manufactured-solution solve, in both
precisions.  The cpu_baseline object times the CPU oracle (plain
NumPy/SciPy FP64) on a bounded sample: V-cycles of the same method at
256 x 256 elements; it also solves the 256 x 256 manufactured problem with
the oracle and reports the GPU solutions' distance to it.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector, published
ROOT = os.path.dirname(os.path.abspath(__file__))


def measured_traffic():
    """HBM bytes per launch of the finest-level Vanka tile kernel measured with rocprofv3 byte
    counters (profiles/vanka_tile_traffic.json), or None if the kernel
    source has changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "vanka_tile_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        with open(os.path.join(ROOT, d["source"]), "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    if h != d.get("kernel_source_sha256"):
        return None
    return float(d["read_bytes"] + d["write_bytes"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-N", type=int, default=256)
    ap.add_argument("--cpu-levels", type=int, default=6)
    ap.add_argument("--cpu-vcycles", type=int, default=60)
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--skip-c2", action="store_true",
                    help="skip the 256x256 sweep and solve measurements")
    ap.add_argument("--skip-c4", action="store_true",
                    help="skip the 512x512 batched (32 right-hand sides) solves")
    ap.add_argument("--c4-batch", type=int, default=32)
    ap.add_argument("--skip-bs", action="store_true",
                    help="skip the Braess-Sarazin comparison solves")
    ap.add_argument("--skip-adjoint", action="store_true",
                    help="skip the forward + adjoint (gradient) timing")
    ap.add_argument("--skip-c5", action="store_true",
                    help="skip the 256x256 per-element viscosity solves and gradients")
    ap.add_argument("--interior-apply", choices=["vector", "matrix"], default="vector",
                    help="interior Vanka apply: vector ALUs (default) or matrix cores")
    ap.add_argument("--vcycle-only", action="store_true",
                    help="only set up the FP64 (and FP32) contexts and time V-cycles: the "
                         "median cycle and the per-level kernel table (for profiling)")
    ap.add_argument("--autotune", action="store_true",
                    help="only measure the launch-shape tuning (vkmg_autotune) of the FP64 and "
                         "FP32 contexts and print it with the V-cycle times it gives")
    ap.add_argument("--fused-sweep-max-n", type=int, default=-1,
                    help="override the tuning: sweeps of levels with 16 <= N <= this fused "
                         "into one launch (0: never); -1: library default")
    ap.add_argument("--cpu-c3", action="store_true",
                    help="also time the oracle at 1024x1024, 8 levels (one V(2,2) cycle, one "
                         "sweep and the full solve) and one right-hand side of the 512x512 "
                         "batch, compared with the GPU's FP64 solutions (a few minutes on "
                         "the host; not part of the default run)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB "
                         "(3 times) and exit: the reference kernel for scaling HBM "
                         "byte counters")
    return ap.parse_args()


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8}))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def copy_bandwidth(torch, mib=1024, reps=10):
    """Usable HBM bandwidth: read + write bytes per second of a plain device
    copy of `mib` MiB (larger than the 256 MB last-level cache)."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2 * n * 8 / t


def vcycle_roofline(N, L, bw):
    """Time bound of one FP64 V(2,2) cycle: the sum over its kernels of the
    larger of algorithmic bytes / bw and algorithmic flops / the FP64 vector
    peak.  Per relaxed level (n_l DoFs, N_l^2 elements, (N_l+1)^2 patches):
    four Vanka updates (read r and x, write x; the first, from x = 0, does
    not read x; 2*495 + 297 + 51 flops per interior patch in the symmetry
    form, 2*51*51 per boundary patch), four residuals (read x and b, write
    r; about 345 flops per element), the restriction (read n_l, write
    n_{l-1}) and the prolongation (read n_{l-1} and n_l, write n_l); the
    coarse solve reads its n_0 x n_0 inverse."""
    def n_of(Nl):
        return 2 * (2 * Nl + 1) ** 2 + (Nl + 1) ** 2

    peak = FP64_VECTOR_PEAK_TFLOPS * 1e12
    terms = []
    for l in range(1, L):
        Nl = N >> (L - 1 - l)
        n, nc = n_of(Nl), n_of(Nl // 2)
        pb = 8 * Nl - 8
        pint = (Nl + 1) ** 2 - pb
        fv = pint * (2 * 495 + 297 + 51) + pb * 2 * 51 * 51
        for k in range(4):
            terms.append((("vanka", Nl), (16 if k == 0 else 24) * n, fv))
            terms.append((("residual", Nl), 24 * n, 345 * Nl * Nl))
        terms.append((("restrict", Nl), 8 * (n + nc), 20 * Nl * Nl))
        terms.append((("prolong", Nl), 8 * (nc + 2 * n), 20 * Nl * Nl))
    n0 = n_of(N >> (L - 1)) + 1
    terms.append((("coarse", N >> (L - 1)), 8 * n0 * n0, 2 * n0 * n0))
    t_roof = sum(max(b / bw, f / peak) for _, b, f in terms)
    nbytes = sum(b for _, b, _ in terms)
    flops = sum(f for _, _, f in terms)
    return t_roof, nbytes, flops


def vcycle_level_table(s, vk, torch, r, z, N, L, reps=20):
    """Kernel time per V-cycle by level and kernel class, from HIP events
    around every launch on the cycle's stream (launch by launch, no graph)."""
    classes = {"vanka": vk.KERNEL_VANKA, "residual": vk.KERNEL_RESIDUAL,
               "transfer": vk.KERNEL_TRANSFER, "coarse": vk.KERNEL_COARSE}
    s.set_timing(sum(1 << c for c in classes.values()))
    for _ in range(reps):
        s.vcycle(r, z)
    torch.cuda.synchronize()
    rows = []
    for l in range(L - 1, -1, -1):
        row = {"level": l, "N": N >> (L - 1 - l)}
        tot = 0.0
        for k, c in classes.items():
            n, ms = s.kernel_timing(c, l)
            if n:
                row[f"{k}_us"] = round(ms * 1e3 / reps, 2)
                row[f"{k}_launches"] = n // reps
                tot += ms * 1e3 / reps
        row["total_us"] = round(tot, 2)
        rows.append(row)
    s.set_timing(0)
    return rows


def timed_vcycles(s, torch, r, z, reps=20, warm=5):
    """Median of `reps` V-cycles (HIP events around each on the current stream)."""
    for _ in range(warm):
        s.vcycle(r, z)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s.vcycle(r, z)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def vcycle_only(a):
    """Set up the benchmark's contexts and time V-cycles only (for
    profiling): median cycle in both precisions and the per-level table."""
    import torch

    import paper_2401_06277_amd as vk
    from stokes_inputs import uniform_vector, velocity_dirichlet_mask

    torch.cuda.set_device(0)
    N, L = a.N, a.levels
    out = {"N": N, "levels": L}
    for prec in ("fp64", "fp32"):
        log(f"[bench] V-cycles {prec}")
        s = vk.VkmgSolver(N, L, precision=prec, interior_apply=a.interior_apply)
        if a.fused_sweep_max_n >= 0:
            s.set_tuning(fused_sweep_max_n=a.fused_sweep_max_n)
        out[f"tuning_{prec}"] = s.get_tuning()
        n = s.layout["n"]
        rh = uniform_vector(n, 170)
        rh[velocity_dirichlet_mask(N)] = 0.0
        r = torch.from_numpy(rh).cuda()
        z = torch.empty_like(r)
        out[f"vcycle_s_{prec}"] = timed_vcycles(s, torch, r, z)
        out[f"levels_{prec}"] = vcycle_level_table(s, vk, torch, r, z, N, L)
        s.close()
    print(json.dumps(out), flush=True)


def autotune_only(a):
    """Run the library's autotuner on the benchmark's FP64 and FP32
    contexts; print the chosen launch shapes and the median V-cycle under
    the library defaults, with every fusion off, and under the tuned
    choice."""
    import torch

    import paper_2401_06277_amd as vk
    from stokes_inputs import uniform_vector, velocity_dirichlet_mask

    torch.cuda.set_device(0)
    N, L = a.N, a.levels
    never = 2**31 - 1
    plain = dict(fused_sweep_max_n=0, park_min_n=never, fused_prolong_max_n=0,
                 boundary_per_wave=1)
    out = {"N": N, "levels": L}
    for prec in ("fp64", "fp32"):
        log(f"[bench] autotune {prec}")
        s = vk.VkmgSolver(N, L, precision=prec)
        n = s.layout["n"]
        rh = uniform_vector(n, 170)
        rh[velocity_dirichlet_mask(N)] = 0.0
        r = torch.from_numpy(rh).cuda()
        z = torch.empty_like(r)
        default = s.get_tuning()
        t_default = timed_vcycles(s, torch, r, z)
        s.set_tuning(**plain)
        t_plain = timed_vcycles(s, torch, r, z)
        s.set_tuning(**default)
        t0 = time.perf_counter()
        tuned = s.autotune(reps=10)
        t_tune = time.perf_counter() - t0
        t_tuned = timed_vcycles(s, torch, r, z)
        out[prec] = {"default": default, "vcycle_s_default": t_default,
                     "plain": plain, "vcycle_s_plain": t_plain,
                     "tuned": tuned, "vcycle_s_tuned": t_tuned, "autotune_s": t_tune,
                     "levels": vcycle_level_table(s, vk, torch, r, z, N, L)}
        s.close()
    print(json.dumps(out), flush=True)


def cpu_baseline_c3(x_gpu=None, it_gpu=None):
    """The oracle at 1024 x 1024, 8 levels, on the host cores: the
    hierarchy's setup, one V(2,2) cycle, one finest-level sweep (residual and
    update) and the update alone, and the full FGMRES(30) solve to 1e-8 from
    x0 = 0; with the GPU's FP64 solution, its distance to the oracle's (the
    pressure constant removed)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import fem, fgmres, multigrid
    from stokes_inputs import gaussian_random_field

    N, L = 1024, 8
    t0 = time.perf_counter()
    H = multigrid.Hierarchy(N, L, progress=lambda m: log(f"[bench] oracle {m}, "
                                                          f"{time.perf_counter() - t0:.0f} s"))
    setup_s = time.perf_counter() - t0
    f = gaussian_random_field(N, 5, length=0.1)
    _, b, _, _ = fem.stokes_system(N, 1.0, f_nodal=f)
    log("[bench] oracle V-cycle at 1024x1024")
    t0 = time.perf_counter()
    z = H.vcycle(b)
    dt = time.perf_counter() - t0
    lev = H.levels[-1]
    log("[bench] oracle finest-level sweep")
    t0 = time.perf_counter()
    lev.smoother.sweep(z, b)
    sweep_s = time.perf_counter() - t0
    r = b - lev.A @ z
    t0 = time.perf_counter()
    lev.smoother.apply_to_residual(r)
    apply_s = time.perf_counter() - t0
    log("[bench] oracle FGMRES solve at 1024x1024")
    t0 = time.perf_counter()
    res = fgmres.fgmres(H.A, b, np.zeros_like(b), H.vcycle, rtol=1e-8, restart=30, max_iters=100)
    solve_s = time.perf_counter() - t0
    blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    out = {"value": H.patch_updates_per_cycle() / dt, "unit": "patch-updates/s",
           "cores": int(blas_threads), "kind": "oracle",
           "sample": (f"1 FP64 V(2,2) cycle of the oracle at {N}x{N} elements, {L} levels; "
                      "one finest-level sweep; the full FGMRES(30) solve to 1e-8"),
           "seconds_per_vcycle": dt, "setup_s": setup_s,
           "sweep_s": sweep_s, "sweep_patch_updates_per_s": (N + 1) ** 2 / sweep_s,
           "update_only_s": apply_s,
           "solve": {"seconds": solve_s, "iterations": res.iterations,
                     "true_rel_res": float(np.linalg.norm(b - H.A @ res.x) / np.linalg.norm(b))}}
    if x_gpu is not None:
        off_p = 2 * (2 * N + 1) ** 2

        def centred(v):
            v = np.array(v, dtype=np.float64, copy=True)
            v[off_p:] -= v[off_p:].mean()
            return v

        xo = centred(res.x)
        out["solve"]["fp64_gpu_iterations"] = it_gpu
        out["solve"]["fp64_gpu_rel_err_vs_oracle"] = float(
            np.linalg.norm(centred(x_gpu) - xo) / np.linalg.norm(xo))
    return out


def cpu_baseline_c4(gpu=None, batch=32):
    """The oracle's solve of right-hand side 0 of the 512 x 512, 7-level
    batched workload (GRF body force seed 1000, lid u = (1, 0) on the top
    edge, x0 = the Dirichlet lifting, FGMRES(30) to 1e-8), on the host cores,
    setup timed apart; the batch's time extrapolated as `batch` such solves;
    with the GPU's FP64 batched solution of that right-hand side, its distance
    to the oracle's (the pressure constant removed)."""
    import numpy as np

    from oracle import fem, fgmres, multigrid
    from stokes_inputs import gaussian_random_field, lid_boundary_values

    N, L = 512, 7
    t0 = time.perf_counter()
    H = multigrid.Hierarchy(N, L)
    A, b, _, xl = fem.stokes_system(N, 1.0, f_nodal=gaussian_random_field(N, 1000),
                                    g_nodal=lid_boundary_values(N))
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    ro = fgmres.fgmres(A, b, xl, H.vcycle, rtol=1e-8, restart=30, max_iters=500)
    solve_s = time.perf_counter() - t0
    out = {"setup_s": setup_s, "seconds_per_rhs": solve_s, "iterations": ro.iterations,
           f"seconds_for_{batch}_rhs_extrapolated": batch * solve_s,
           "sample": ("one right-hand side of the 512x512, 7-level batch (seed 1000, lid), "
                      f"timed once; the batch as {batch} such solves")}
    if gpu is not None:
        xg, itg = gpu
        off_p = 2 * (2 * N + 1) ** 2

        def centred(v):
            v = np.array(v, dtype=np.float64, copy=True)
            v[off_p:] -= v[off_p:].mean()
            return v

        xo = centred(ro.x)
        out["fp64_gpu_batched_iterations"] = itg
        out["fp64_gpu_batched_rel_err_vs_oracle"] = float(
            np.linalg.norm(centred(xg) - xo) / np.linalg.norm(xo))
    return out


def cpu_baseline(N, levels, nvc, c2=None):
    """Oracle V-cycles at N x N (setup excluded), patch-updates/s.  With the
    256 x 256 GPU solutions, also the oracle's own FGMRES solve of that
    problem and the GPU solutions' distance to it."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import fem, multigrid
    from stokes_inputs import gaussian_random_field

    t0 = time.perf_counter()
    H = multigrid.Hierarchy(N, levels)
    setup_s = time.perf_counter() - t0
    f = gaussian_random_field(N, 5, length=0.1)
    _, b, _, _ = fem.stokes_system(N, 1.0, f_nodal=f)
    H.vcycle(b)  # warm
    t0 = time.perf_counter()
    for _ in range(nvc):
        H.vcycle(b)
    dt = time.perf_counter() - t0
    ups = H.patch_updates_per_cycle() * nvc / dt
    blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    extra = {}
    # the same V-cycles on one thread (the paper's CPU runs are serial)
    from threadpoolctl import threadpool_limits
    n1 = max(nvc // 6, 3)
    with threadpool_limits(limits=1):
        H.vcycle(b)
        t0 = time.perf_counter()
        for _ in range(n1):
            H.vcycle(b)
        dt1 = time.perf_counter() - t0
    extra["single_thread"] = {"value": H.patch_updates_per_cycle() * n1 / dt1,
                              "unit": "patch-updates/s", "cores": 1,
                              "sample": f"{n1} V(2,2) cycles at {N}x{N}, BLAS limited to 1 thread"}
    # C1: the 16 x 16, 3-level manufactured-solution solve, setup included
    from oracle import fgmres
    from stokes_inputs import manufactured_boundary_values, manufactured_nodal_force
    t0 = time.perf_counter()
    H1 = multigrid.Hierarchy(16, 3)
    A1, b1, _, xl1 = fem.stokes_system(16, 1.0, f_nodal=manufactured_nodal_force(16, "trig"),
                                       g_nodal=manufactured_boundary_values(16, "trig"))
    r1 = fgmres.fgmres(A1, b1, xl1, H1.vcycle, rtol=1e-8, restart=30, max_iters=500)
    extra["oracle_solve_16"] = {"seconds": time.perf_counter() - t0, "iterations": r1.iterations,
                                "sample": "16x16 elements, 3 levels, trigonometric manufactured "
                                          "solution, FGMRES(30) to 1e-8, setup included"}
    if c2 is not None and N == 256:
        from oracle import fgmres
        from stokes_inputs import manufactured_boundary_values, manufactured_nodal_force
        gd = manufactured_boundary_values(N, "trig")
        A, bo, _, xl = fem.stokes_system(N, 1.0, f_nodal=manufactured_nodal_force(N, "trig"),
                                         g_nodal=gd)
        t0 = time.perf_counter()
        ro = fgmres.fgmres(A, bo, xl, H.vcycle, rtol=1e-8, restart=30, max_iters=500)
        t_solve = time.perf_counter() - t0
        xo = fem.normalise_pressure(N, ro.x)
        extra["oracle_solve_256"] = {"seconds": t_solve, "iterations": ro.iterations}
        for prec, xg in c2["_solutions"].items():
            xa = fem.normalise_pressure(N, xg.astype(np.float64))
            extra["oracle_solve_256"][f"{prec}_rel_err_vs_oracle"] = float(
                np.linalg.norm(xa - xo) / np.linalg.norm(xo))
            extra["oracle_solve_256"][f"{prec}_iterations"] = c2[f"solve_{prec}"]["iterations"]
    return {
        "value": ups,
        "unit": "patch-updates/s",
        "cores": int(blas_threads),
        "kind": "oracle",
        "sample": (f"{nvc} FP64 V(2,2) cycles of the oracle at {N}x{N} elements, {levels} levels "
                   f"(setup {setup_s:.1f} s excluded, {dt:.1f} s timed); dense BLAS on "
                   f"{blas_threads} threads, sparse matvecs single-threaded; host has "
                   f"{os.cpu_count()} logical CPUs"),
        "seconds_per_vcycle": dt / nvc,
        **extra,
    }


def bench_c2(a, vk, torch, np):
    """256 x 256, 6 levels: standalone sweep rates (apply only, given r; and
    residual + update, given x and b) in both precisions, and the
    manufactured-solution solve (trigonometric solution, Dirichlet lifting
    as initial guess) in both precisions."""
    from stokes_inputs import (dirichlet_consistent_pair, grid_sizes, manufactured_boundary_values,
                               manufactured_nodal_force, uniform_vector, velocity_dirichlet_mask)

    N2, L2 = 256, 6
    g = grid_sizes(N2)
    top = L2 - 1
    mask = velocity_dirichlet_mask(N2)
    rin = uniform_vector(g.n, 2)
    rin[mask] = 0.0
    xin, bin_ = dirichlet_consistent_pair(N2, 3, 4)
    res = {"config": "256x256 elements, 6 levels, V(2,2) omega=0.5; sweeps on the finest level"}

    def timed(fn, reps=20, warm=5):
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        ts.sort()
        return ts[len(ts) // 2]

    fn2 = manufactured_nodal_force(N2, "trig")
    gd2 = manufactured_boundary_values(N2, "trig")
    sol = {}
    for prec in ("fp64", "fp32"):
        dt = torch.float32 if prec == "fp32" else torch.float64
        s = vk.VkmgSolver(N2, L2, precision=prec, interior_apply=a.interior_apply)
        r_d = torch.from_numpy(rin).to(dt).cuda()
        x_d = torch.zeros(g.n, dtype=dt, device="cuda")
        t_apply = timed(lambda: s.vanka_update(top, x_d, r_d))
        x_d = torch.from_numpy(xin).to(dt).cuda()
        b_d = torch.from_numpy(bin_).to(dt).cuda()
        t_full = timed(lambda: s.vanka_sweep(top, x_d, b_d))
        res[f"sweep_apply_only_{prec}"] = {"us": t_apply * 1e6,
                                           "patch_updates_per_s": (N2 + 1) ** 2 / t_apply}
        res[f"sweep_full_{prec}"] = {"us": t_full * 1e6,
                                     "patch_updates_per_s": (N2 + 1) ** 2 / t_full}
        b = s.assemble_rhs(torch.from_numpy(fn2.ravel()).cuda(),
                           torch.from_numpy(gd2.ravel()).cuda())
        x0 = s.dirichlet_lift(b)
        x = x0.clone()
        s.fgmres_solve(b, x, rtol=1e-8)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = x0.clone()
        info = s.fgmres_solve(b, x, rtol=1e-8)
        torch.cuda.synchronize()
        res[f"solve_{prec}"] = {"time_to_1e8_s": time.perf_counter() - t0,
                                "iterations": info["iterations"],
                                "true_rel_res": info["true_rel_res"]}
        sol[prec] = x.cpu().numpy()
        s.close()
    res["_solutions"] = sol
    return res


def bench_c4(a, vk, torch, np):
    """512 x 512, 7 levels, B = 32 right-hand sides: Gaussian random body
    forces (unit variance, l = 0.1, seeds 1000 + k) under the lid-driven top
    boundary, solved to rtol 1e-8 as one batched FGMRES (batched context)
    and as B sequential single-right-hand-side solves, FP32 and FP64
    multigrid.  Times exclude setup and the right-hand-side assembly."""
    from concurrent.futures import ThreadPoolExecutor

    from stokes_inputs import gaussian_random_field, lid_boundary_values

    N4, L4, B = 512, 7, a.c4_batch
    with ThreadPoolExecutor(8) as ex:
        fs = list(ex.map(lambda k: gaussian_random_field(N4, 1000 + k).ravel(), range(B)))
    g = lid_boundary_values(N4).ravel()
    ups = sum(4 * ((N4 >> (L4 - 1 - l)) + 1) ** 2 for l in range(1, L4))
    res = {"config": (f"512x512 elements, 7 levels, {B} right-hand sides (GRF body force l=0.1 "
                      "seeds 1000+k, lid u=(1,0) on the top edge), FGMRES(30) rtol 1e-8, "
                      "x0 = Dirichlet lifting"),
           "batch": B, "patch_updates_per_vcycle_per_rhs": ups}
    fd = torch.from_numpy(np.concatenate(fs)).cuda()
    gd = torch.from_numpy(np.tile(g, B)).cuda()
    for prec in ("fp32", "fp64"):
        log(f"[bench] 512x512 x{B} batched {prec}")
        s = vk.VkmgSolver(N4, L4, precision=prec, interior_apply=a.interior_apply, batch=B)
        n = s.layout["n"]
        b = s.assemble_rhs(fd, gd)
        x0 = s.dirichlet_lift(b)
        x = x0.clone()
        s.fgmres_solve(b, x, rtol=1e-8, restart=30, max_iters=500)  # warm (captures graphs)
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = s.fgmres_solve(b, x, rtol=1e-8, restart=30, max_iters=500)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        its = [i["iterations"] for i in infos]
        xb = x.view(B, n)
        res[f"batched_{prec}"] = {
            "time_s": tb, "time_per_rhs_s": tb / B,
            "iterations_max": max(its), "iterations_mean": sum(its) / B,
            "max_true_rel_res": max(i["true_rel_res"] for i in infos),
            "all_converged": all(i["status_name"] == "VKMG_OK" for i in infos),
            "patch_updates_per_s": ups * sum(its) / tb,
        }
        s.close()
        log(f"[bench] 512x512 x{B} sequential {prec}")
        s1 = vk.VkmgSolver(N4, L4, precision=prec, interior_apply=a.interior_apply)
        bs = [s1.assemble_rhs(fd[k * len(g):(k + 1) * len(g)], gd[:len(g)]) for k in range(B)]
        x1 = s1.dirichlet_lift(bs[0])
        s1.fgmres_solve(bs[0], x1, rtol=1e-8, restart=30, max_iters=500)  # warm
        xs, its1 = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(B):
            x1 = s1.dirichlet_lift(bs[k])
            info = s1.fgmres_solve(bs[k], x1, rtol=1e-8, restart=30, max_iters=500)
            its1.append(info["iterations"])
            xs.append(x1)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        off_p = 2 * (2 * N4 + 1) ** 2

        def centred(v):
            v = v.clone()
            v[off_p:] -= v[off_p:].mean()
            return v

        dmax = max(float(torch.linalg.norm(centred(xb[k]) - centred(xs[k]))
                         / torch.linalg.norm(centred(xs[k]))) for k in range(B))
        res[f"sequential_{prec}"] = {"time_s": ts, "time_per_rhs_s": ts / B,
                                     "iterations_max": max(its1),
                                     "patch_updates_per_s": ups * sum(its1) / ts}
        res[f"batched_speedup_{prec}"] = ts / tb
        res[f"batched_vs_sequential_max_rel_diff_{prec}"] = dmax
        if prec == "fp64":  # right-hand side 0, for the oracle comparison
            res["_solution_fp64_rhs0"] = (xb[0].cpu().numpy(), its[0])
        s1.close()
        del xs, bs, b, x, x0, xb
        torch.cuda.empty_cache()
    return res


def bench_bs(a, vk, torch, fd, N, L, vanka_ms):
    """Braess-Sarazin relaxation (t = 1, omega_bs = 1, Jacobi weight 1, two
    Jacobi sweeps) in the same V(2,2)-preconditioned FGMRES on the headline
    workload, FP64 and FP32 multigrid, against the Vanka solves timed above;
    relaxation time per finest-level sweep from HIP events."""
    res = {"config": "inexact Braess-Sarazin, t=1, omega_bs=1, Jacobi weight 1, 2 Jacobi sweeps "
                     "on S; same V(2,2) cycle, FGMRES(30), rtol 1e-8, workload as above"}
    for prec in ("fp64", "fp32"):
        log(f"[bench] braess-sarazin {prec}")
        s = vk.VkmgSolver(N, L, precision=prec, relaxation="braess_sarazin")
        b = s.assemble_rhs(fd)
        x = torch.zeros_like(b)
        s.fgmres_solve(b, x, rtol=a.rtol)  # warm (captures graphs)
        ts, its, infos = [], [], []
        for _ in range(max(a.steps, 2)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.fgmres_solve(b, x, rtol=a.rtol, restart=30, max_iters=500)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            its.append(info["iterations"])
            infos.append(info)
        s.set_timing(1 << vk.KERNEL_VANKA)
        x.zero_()
        s.fgmres_solve(b, x, rtol=a.rtol, restart=30, max_iters=500)
        nl, ms = s.kernel_timing(vk.KERNEL_VANKA, L - 1)
        s.set_timing(0)
        ts.sort()
        t_med = ts[len(ts) // 2]
        res[prec] = {"time_to_1e8_s": t_med, "fgmres_iterations": its[0],
                     "true_rel_res": infos[-1]["true_rel_res"],
                     "converged": all(i["status_name"] == "VKMG_OK" for i in infos),
                     "relaxation_us_per_finest_sweep": ms / max(nl, 1) * 1e3}
        if prec in vanka_ms:
            res[prec]["vanka_time_to_1e8_s"] = vanka_ms[prec]
            res[prec]["vanka_over_bs_time"] = vanka_ms[prec] / t_med
        s.close()
        # Vanka with the damping that minimises its iteration count in the
        # oracle's study (0.7-0.8), for a comparison of tuned schemes
        log(f"[bench] vanka omega=0.75 {prec}")
        s = vk.VkmgSolver(N, L, precision=prec, omega=0.75, interior_apply=a.interior_apply)
        b = s.assemble_rhs(fd)
        x = torch.zeros_like(b)
        s.fgmres_solve(b, x, rtol=a.rtol)
        ts = []
        for _ in range(max(a.steps, 2)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.fgmres_solve(b, x, rtol=a.rtol, restart=30, max_iters=500)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        res[prec]["vanka_omega075_time_to_1e8_s"] = ts[len(ts) // 2]
        res[prec]["vanka_omega075_iterations"] = info["iterations"]
        s.close()
    return res


def bench_adjoint(a, vk, torch, fd, N, L):
    """Gradient of L = |x - x_t|^2 / 2 with respect to the body force on the
    headline workload: forward solve + adjoint solve + transposed load map
    (paper_2401_06277_amd.autograd), FP64 multigrid, rtol 1e-8 both ways."""
    import numpy as np

    from paper_2401_06277_amd.autograd import stokes_solve
    from stokes_inputs import gaussian_random_field

    log("[bench] adjoint (force gradient)")
    s = vk.VkmgSolver(N, L)
    xt = torch.from_numpy(np.ascontiguousarray(
        np.concatenate([gaussian_random_field(N, 6).ravel(),
                        np.zeros((N + 1) ** 2)]))).cuda() * 0.01
    ts = []
    for k in range(max(a.steps, 2) + 1):
        f = fd.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = stokes_solve(f, s, rtol=a.rtol)
        loss = 0.5 * torch.sum((x - xt) ** 2)
        loss.backward()
        torch.cuda.synchronize()
        if k > 0:  # the first pass captures the graphs
            ts.append(time.perf_counter() - t0)
    ts.sort()
    s.close()
    return {"config": "L = |x - x_t|^2/2, x_t = 0.01 GRF (seed 6) on the velocity, rtol 1e-8; "
                      "forward + backward wall time",
            "time_s": ts[len(ts) // 2],
            "grad_norm": float(torch.linalg.norm(f.grad))}


def bench_c5(a, vk, torch, np):
    """256 x 256, 6 levels, per-element viscosity log nu_e ~ U[-1,1] (seed 7):
    setup (per-patch inverses on the host threads), FGMRES solve to 1e-8
    with "simple" Vanka (one stored inverse per patch), and the gradient of
    L = |x - x_t|^2 / 2 (x_t: GRF seed 6 on the velocity) with respect to the
    force and the viscosity (forward + adjoint); the constant-viscosity
    solve of the same problem for comparison."""
    from paper_2401_06277_amd.autograd import stokes_solve
    from stokes_inputs import gaussian_random_field, log_viscosity_field

    N5, L5 = 256, 6
    nu = np.exp(log_viscosity_field(N5, 7))
    f = torch.from_numpy(np.ascontiguousarray(gaussian_random_field(N5, 5).ravel())).cuda()
    xt = torch.from_numpy(np.ascontiguousarray(np.concatenate(
        [gaussian_random_field(N5, 6).ravel(), np.zeros((N5 + 1) ** 2)]))).cuda() * 0.01
    res = {"config": "256x256 elements, 6 levels, log nu_e ~ U[-1,1] (seed 7), GRF force (seed 5), "
                     "FGMRES(30) + V(2,2) simple Vanka omega=0.5, rtol 1e-8; loss |x - x_t|^2/2"}
    for label, kw in (("variable_nu", {"nu_elem": nu}), ("constant_nu", {})):
        log(f"[bench] 256x256 {label}")
        t0 = time.perf_counter()
        s = vk.VkmgSolver(N5, L5, **kw)
        setup = time.perf_counter() - t0
        b = s.assemble_rhs(f)
        x = torch.zeros_like(b)
        s.fgmres_solve(b, x, rtol=1e-8)
        ts = []
        for _ in range(max(a.steps, 2)):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.fgmres_solve(b, x, rtol=1e-8)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        res[label] = {"setup_s": setup, "time_to_1e8_s": ts[len(ts) // 2],
                      "iterations": info["iterations"], "true_rel_res": info["true_rel_res"]}
        if label == "variable_nu":
            nud = torch.from_numpy(nu).cuda()
            tg = []
            for k in range(3):
                fd = f.clone().requires_grad_(True)
                nv = nud.clone().requires_grad_(True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xs = stokes_solve(fd, s, nu=nv, rtol=1e-8)
                (0.5 * torch.sum((xs - xt) ** 2)).backward()
                torch.cuda.synchronize()
                if k > 0:
                    tg.append(time.perf_counter() - t0)
            res[label]["forward_backward_s"] = min(tg)
            res[label]["grad_nu_norm"] = float(torch.linalg.norm(nv.grad))
        s.close()
    return res


def main():
    a = parse()
    if a.copy_calibration_mib:
        copy_calibration(a.copy_calibration_mib)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are "
                                   "not supported (use --gpus 1)"}))
        sys.exit(2)
    if a.vcycle_only:
        vcycle_only(a)
        return
    if a.autotune:
        autotune_only(a)
        return
    import numpy as np
    import torch

    import paper_2401_06277_amd as vk
    from stokes_inputs import gaussian_random_field

    torch.cuda.set_device(0)
    N, L = a.N, a.levels
    log(f"[bench] setup N={N} levels={L}")
    f = gaussian_random_field(N, 5, length=0.1)
    fd = torch.from_numpy(np.ascontiguousarray(f.ravel())).cuda()

    def make(prec):
        s = vk.VkmgSolver(N, L, precision=prec, interior_apply=a.interior_apply)
        if a.fused_sweep_max_n >= 0:
            s.set_tuning(fused_sweep_max_n=a.fused_sweep_max_n)
        b = s.assemble_rhs(fd)
        x = torch.zeros_like(b)
        return s, b, x

    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    s64, b, x = make("fp64")
    torch.cuda.synchronize()
    setup64_s = time.perf_counter() - t_setup  # vkmg_setup and the load assembly
    n = s64.layout["n"]
    ups_per_cycle = sum(4 * ((N >> (L - 1 - l)) + 1) ** 2 for l in range(1, L))

    def run_solves(s, b, x, steps, timed):
        iters = []
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            info = s.fgmres_solve(b, x, rtol=a.rtol, restart=30, max_iters=500)
            iters.append(info["iterations"])
            infos.append(info)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, iters, infos

    log("[bench] fp64 warmup")
    run_solves(s64, b, x, a.warmup, False)
    log("[bench] fp64 timed")
    dt64, it64, inf64 = run_solves(s64, b, x, a.steps, True)
    # kernel durations: HIP events around every finest-level Vanka update on
    # the solve's stream, in a second pass of the same solves (events bypass
    # the captured graphs, so this pass launches kernel by kernel)
    log("[bench] fp64 event-timed pass")
    classes = {"vanka": vk.KERNEL_VANKA, "residual": vk.KERNEL_RESIDUAL,
               "transfer": vk.KERNEL_TRANSFER, "coarse": vk.KERNEL_COARSE,
               "krylov": vk.KERNEL_KRYLOV}
    s64.set_timing(sum(1 << c for c in classes.values()) | (1 << vk.KERNEL_VANKA_TILE))
    dt64_ev, _, _ = run_solves(s64, b, x, a.steps, True)
    nl, ms = s64.kernel_timing(vk.KERNEL_VANKA, L - 1)
    nt, ms_tile = s64.kernel_timing(vk.KERNEL_VANKA_TILE, L - 1)
    breakdown = {k: s64.kernel_timing(c)[1] / a.steps for k, c in classes.items()}
    s64.set_timing(0)
    for inf in inf64:
        if inf["status_name"] != "VKMG_OK":
            log(f"[bench] solve did not converge: {inf}")
            sys.exit(1)
    x64 = x.clone()
    value = ups_per_cycle * sum(it64) / dt64
    # algorithmic bytes of the finest-level updates, 8 bytes per scalar: each
    # reads the residual and writes the iterate over all n DoFs, and reads
    # the iterate too except in the first pre-smoothing sweep of a cycle,
    # which starts from x = 0 (16 n bytes there, 24 n elsewhere); V(2,2):
    # 4 updates per cycle, 22 n bytes per launch on average
    per_cycle = 4
    assert nl % per_cycle == 0 and nt == nl, (nl, nt)
    alg_bytes_total = nl // per_cycle * (16 + 24 * (per_cycle - 1)) * n
    alg_bytes = alg_bytes_total / nl
    avg_tile_s = ms_tile / 1e3 / max(nt, 1)
    avg_launch_s = ms / 1e3 / max(nl, 1)
    achieved = alg_bytes / avg_tile_s / 1e9
    achieved_update = alg_bytes / avg_launch_s / 1e9

    # standalone V-cycle rate (median of 20)
    r = torch.randn(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    for _ in range(5):
        s64.vcycle(r, z)
    ts = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s64.vcycle(r, z)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    ts.sort()
    vcycle_s = ts[len(ts) // 2]
    del r, z
    bw = copy_bandwidth(torch)
    t_roof, vc_bytes, vc_flops = vcycle_roofline(N, L, bw)

    out = {
        "metric": "Vanka V-cycle patch-updates/s + FGMRES time-to-1e-8, FP64 vs FP32-MG, 1024²",
        "value": value,
        "unit": "patch-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt64 / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"2D Stokes Q2-Q1, {N}x{N} elements, {L} levels, GRF body force "
                         f"(l=0.1, seed 5), FGMRES(30) + V(2,2) Vanka omega=0.5, rtol {a.rtol:g}"),
            "N": N, "levels": L, "dofs": n, "patch_updates_per_vcycle": ups_per_cycle,
            "interior_apply": a.interior_apply,
            "tuning": s64.get_tuning(),
        },
        "time_to_1e8_s": dt64 / a.steps,
        "setup_s": setup64_s,
        "time_to_1e8_s_without_graphs": dt64_ev / a.steps,
        "kernel_ms_per_solve": breakdown,
        "krylov_share": breakdown["krylov"] / max(sum(breakdown.values()), 1e-300),
        "fgmres_iterations": it64[0],
        "true_rel_res": inf64[-1]["true_rel_res"],
        "vcycle_s": vcycle_s,
        "vcycle_patch_updates_per_s": ups_per_cycle / vcycle_s,
        "vcycle_roofline": {
            "t_roof_s": t_roof,
            "frac": t_roof / vcycle_s,
            "alg_bytes": vc_bytes,
            "alg_flops": vc_flops,
            "hbm_frac_of_copy": vc_bytes / vcycle_s / bw,
            "hbm_frac_of_peak": vc_bytes / vcycle_s / (HBM_PEAK_GBS * 1e9),
            "copy_bandwidth_gbs": bw / 1e9,
            "model": "sum over the cycle's kernels of max(algorithmic bytes / measured copy "
                     "bandwidth, algorithmic flops / FP64 vector peak); launch latency not "
                     "modelled",
        },
        "roofline": {
            "kernel": ("interior-tile kernel of the finest-level Vanka update ("
                       + ("vanka_mfma_kernel" if a.interior_apply == "matrix"
                          else "vanka_sweep_kernel<double,false,true>") + ")"),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "launches": nt,
            "avg_launch_us": avg_tile_s * 1e6,
            "alg_bytes_per_launch": alg_bytes,
            "alg_bytes_rule": "16 n bytes for the update from x = 0 (first pre-smoothing "
                              "sweep), 24 n for the other three of each V(2,2) cycle; "
                              "n = DoFs of the finest level",
            "timing": "HIP events around each finest-level tile-kernel launch on the solve "
                      "stream, event-timed pass of the same solves",
            "with_boundary_kernel": {
                "avg_launch_us": avg_launch_s * 1e6,
                "achieved": achieved_update,
                "frac": achieved_update / HBM_PEAK_GBS,
            },
        },
    }
    s64.close()

    if not a.skip_fp32:
        torch.cuda.synchronize()
        t_setup = time.perf_counter()
        s32, b32, x32 = make("fp32")
        torch.cuda.synchronize()
        setup32_s = time.perf_counter() - t_setup
        log("[bench] fp32-mg warmup")
        run_solves(s32, b32, x32, a.warmup, False)
        log("[bench] fp32-mg timed")
        dt32, it32, inf32 = run_solves(s32, b32, x32, a.steps, True)
        off_p = 2 * (2 * N + 1) ** 2

        def centred(v):  # remove the pressure constant (the null space)
            v = v.clone()
            v[off_p:] -= v[off_p:].mean()
            return v

        diff = float(torch.linalg.norm(centred(x32) - centred(x64)) / torch.linalg.norm(centred(x64)))
        out["fp32_mg"] = {
            "time_to_1e8_s": dt32 / a.steps,
            "setup_s": setup32_s,
            "fgmres_iterations": it32[0],
            "true_rel_res": inf32[-1]["true_rel_res"],
            "patch_updates_per_s": ups_per_cycle * sum(it32) / dt32,
            "rel_diff_vs_fp64_path": diff,
            "speedup_vs_fp64": dt64 / dt32,
            "converged": all(i["status_name"] == "VKMG_OK" for i in inf32),
        }
        s32.close()

    c2 = None
    if not a.skip_c2:
        log("[bench] 256x256 sweeps and solves")
        c2 = bench_c2(a, vk, torch, np)
        out["c2_256"] = {k: v for k, v in c2.items() if not k.startswith("_")}

    if not a.skip_bs:
        vms = {"fp64": out["time_to_1e8_s"]}
        if "fp32_mg" in out:
            vms["fp32"] = out["fp32_mg"]["time_to_1e8_s"]
        out["braess_sarazin"] = bench_bs(a, vk, torch, fd, N, L, vms)

    if not a.skip_adjoint:
        out["adjoint_force_gradient"] = bench_adjoint(a, vk, torch, fd, N, L)
        out["adjoint_force_gradient"]["over_forward_solve"] = (
            out["adjoint_force_gradient"]["time_s"] / out["time_to_1e8_s"])

    if not a.skip_c5:
        out["c5_256_variable_viscosity"] = bench_c5(a, vk, torch, np)

    c4 = None
    if not a.skip_c4:
        c4 = bench_c4(a, vk, torch, np)
        out["c4_512_batched"] = {k: v for k, v in c4.items() if not k.startswith("_")}

    if not a.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(a.cpu_N, a.cpu_levels, a.cpu_vcycles, c2)
        if a.cpu_c3:
            log("[bench] cpu baseline at 1024x1024 (oracle: V-cycle, sweep, solve)")
            out["cpu_baseline"]["c3_1024"] = cpu_baseline_c3(x64.cpu().numpy(), it64[0])
            log("[bench] cpu baseline at 512x512, one right-hand side (oracle solve)")
            out["cpu_baseline"]["c4_512"] = cpu_baseline_c4(
                c4.get("_solution_fp64_rhs0") if c4 else None, a.c4_batch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
