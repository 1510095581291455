/*
 * vkmg.h -- Vanka-multigrid preconditioned FGMRES for the structured-grid
 * Q2-Q1 (Taylor-Hood) Stokes discretisation, on one AMD Instinct MI355X.
 *
 * C ABI.  Every vector argument is caller-owned HIP device memory on the
 * device that was current when the context was created, unless stated
 * otherwise; the library owns only its workspace (allocated in
 * vkmg_setup, freed in vkmg_destroy).  No C++ exception and no process
 * exit crosses this interface: every entry point returns a status code and
 * leaves a thread-local message behind (vkmg_last_error).  Arguments are
 * validated before any GPU work is enqueued; on error the outputs are
 * unspecified and the context stays usable.  A context is not thread-safe.
 *
 * Problem (paper, section "Problem setup" and "Discretization"):
 *   -nu lap u + grad p = f, div u = 0 on the unit square, uniform N x N
 *   quadrilateral mesh, biquadratic continuous velocity, bilinear continuous
 *   pressure, Dirichlet velocity data on every edge, pressure defined up to
 *   a constant.  The linear system is the saddle-point matrix
 *   A = [[L, B^T], [B, 0]] (equation "stokesmatrix"), with
 *   b(v, q) = -int q div v, after symmetric elimination of the Dirichlet
 *   DoFs (identity rows and columns on them).
 *
 * Vector layout (every vector, every level): [u_x | u_y | p], where u_x and
 * u_y hold the (2N+1)^2 Q2 nodal values and p the (N+1)^2 Q1 nodal values,
 * each block row-major with flat index j*side + i (i along x).  Q2 node
 * (i,j) sits at (i/(2N), j/(2N)); Q1 node (i,j) at (i/N, j/N).  Dirichlet
 * DoFs (both velocity components at every boundary Q2 node) are present in
 * the vector; their rows are identity rows.
 *
 * Streams: every entry point that takes `stream` (a hipStream_t, NULL =
 * the legacy default stream) enqueues all its GPU work on it.
 * vkmg_residual, vkmg_apply, vkmg_vanka_sweep, vkmg_vanka_update, vkmg_relax, vkmg_restrict,
 * vkmg_prolong_add, vkmg_coarse_solve, vkmg_vcycle and vkmg_assemble_rhs are
 * asynchronous; vkmg_fgmres_solve synchronises (one small device-to-host
 * copy per Arnoldi step) and its vkmg_info is valid on return.
 */
#ifndef VKMG_H
#define VKMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vkmg_ctx vkmg_ctx; /* opaque, library-owned */

typedef enum {
    VKMG_OK = 0,
    VKMG_ERR_INVALID_ARG = 1,    /* NULL pointer, bad size, level out of range */
    VKMG_ERR_UNSUPPORTED = 2,    /* valid request this build does not handle */
    VKMG_ERR_OUT_OF_MEMORY = 3,  /* device or host allocation failed */
    VKMG_ERR_HIP = 4,            /* a HIP runtime call failed (message says which) */
    VKMG_ERR_SINGULAR_PATCH = 5, /* a Vanka patch or the coarse matrix is singular */
    VKMG_ERR_NOT_CONVERGED = 6,  /* FGMRES hit max_iters above the tolerance */
    VKMG_ERR_NONFINITE = 7,      /* NaN/Inf met in the right-hand side or a residual */
    VKMG_STATUS_FORCE_INT32 = 0x7fffffff /* not a status: keeps the type 32-bit and makes every
                                            non-negative int a valid value of it */
} vkmg_status;

typedef enum { VKMG_FP64 = 0, VKMG_FP32 = 1, VKMG_PRECISION_FORCE_INT32 = 0x7fffffff } vkmg_precision;

/* How the interior Vanka patches (all patches two or more elements from the
 * boundary, which share one inverse) are applied: one patch per lane on the
 * vector ALUs (default, the faster on MI355X), or as 16-patch dense
 * products on the matrix cores.  Both give the same result up to rounding
 * order. */
typedef enum {
    VKMG_APPLY_VECTOR = 0,
    VKMG_APPLY_MATRIX = 1,
    VKMG_APPLY_FORCE_INT32 = 0x7fffffff
} vkmg_interior_apply;

/* Relaxation inside the V-cycle: additive Vanka (paper, "Vanka relaxation
 * scheme", Algorithm 3; default) or inexact Braess-Sarazin (paper,
 * "Braess-Sarazin relaxation scheme", Algorithm 2): with D = diag(L) and
 * S = -(1/t) B D^{-1} B^T, weighted-Jacobi sweeps on
 * S dp = r_p - (1/t) B D^{-1} r_u from dp = 0, du = (1/t) D^{-1}(r_u - B^T dp),
 * x += omega_bs (du, dp). */
typedef enum {
    VKMG_RELAX_VANKA = 0,
    VKMG_RELAX_BRAESS_SARAZIN = 1,
    VKMG_RELAX_FORCE_INT32 = 0x7fffffff
} vkmg_relaxation;

typedef struct {
    int32_t nx, ny; /* elements per side on [0,1]^2; nx == ny required */
} vkmg_grid;

typedef struct {
    int32_t nu_pre;              /* Vanka sweeps before the coarse correction (default 2) */
    int32_t nu_post;             /* Vanka sweeps after it (default 2) */
    double omega;                /* Vanka damping (default 0.5) */
    vkmg_precision mg_precision; /* arithmetic of the whole V-cycle (default FP64) */
    vkmg_interior_apply interior_apply; /* default VKMG_APPLY_VECTOR */
    int32_t use_graphs;          /* 1 (default): vkmg_fgmres_solve replays each Arnoldi step
                                    (V-cycle, A z, Gram-Schmidt kernels) as a HIP graph
                                    captured at its first use; 0: direct launches.  Graphs
                                    are bypassed while kernel timing is enabled (events in
                                    a replayed graph cannot be read back). */
    int32_t batch;               /* right-hand sides handled together (1..64, default 1);
                                    see "Batches" below */
    vkmg_relaxation relaxation;  /* default VKMG_RELAX_VANKA */
    double bs_t;                 /* Braess-Sarazin: scaling t of D (> 0, default 1) */
    double bs_omega;             /* Braess-Sarazin: damping omega_bs (0, 2], default 1 */
    double bs_jacobi_weight;     /* Braess-Sarazin: Jacobi weight on S (0, 2], default 1 */
    int32_t bs_jacobi_sweeps;    /* Braess-Sarazin: Jacobi sweeps on S (1..16, default 2) */
} vkmg_options;

typedef struct {
    int64_t n, n_vel, n_pres;    /* total, velocity (both components), pressure DoFs */
    int64_t off_ux, off_uy, off_p;
    int32_t q2_side, q1_side;    /* 2N+1 and N+1 */
    int32_t n_elem;              /* N */
} vkmg_layout;

typedef struct {
    int32_t iterations;          /* Arnoldi steps taken (= preconditioner applications) */
    int32_t restarts;            /* completed restart cycles */
    double est_rel_res;          /* rotated residual estimate / ||b - A x0|| at exit */
    double true_rel_res;         /* recomputed ||b - A x|| / ||b - A x0|| at exit */
    vkmg_status status;          /* VKMG_OK or VKMG_ERR_NOT_CONVERGED / NONFINITE */
} vkmg_info;

/* Kernel classes that vkmg_kernel_timing reports. */
typedef enum {
    VKMG_KERNEL_VANKA = 0,       /* relaxation update: Vanka (gather, patch-inverse apply,
                                    scatter) or Braess-Sarazin (Schur Jacobi, update) */
    VKMG_KERNEL_RESIDUAL = 1,    /* stencil residual / operator apply */
    VKMG_KERNEL_TRANSFER = 2,    /* restriction and prolongation */
    VKMG_KERNEL_COARSE = 3,      /* coarsest-level dense solve */
    VKMG_KERNEL_KRYLOV = 4,      /* FGMRES vector kernels */
    VKMG_KERNEL_VANKA_TILE = 5,  /* the interior-tile kernel of a Vanka update alone (the
                                    boundary-patch kernel before it excluded); constant-
                                    viscosity Vanka only */
    VKMG_KERNEL_COUNT = 6,
    VKMG_KERNEL_FORCE_INT32 = 0x7fffffff
} vkmg_kernel_class;

/*
 * Batches.  A context set up with batch = B > 1 treats B independent
 * right-hand sides of the same operator together: every vector argument
 * of the entry points below then holds B vectors of that argument's size,
 * back to back (right-hand side k at offset k times the single size; for
 * vkmg_assemble_rhs f and g hold B blocks of 2 (2N+1)^2 values), and one
 * kernel launch serves all B (so the coarse levels, whose single launches
 * cannot fill the GPU, do B times the work per launch).  The results equal
 * those of B separate single-right-hand-side calls up to rounding order.
 */

/* {2, 2, 0.5, VKMG_FP64, VKMG_APPLY_VECTOR, 1, 1, VKMG_RELAX_VANKA, 1, 1, 1, 2}:
 * V(2,2) cycles of additive Vanka damped by 0.5, one right-hand side. */
vkmg_options vkmg_default_options(void);

/*
 * Build the multigrid hierarchy for the Stokes operator with constant
 * viscosity nu on an nx x nx mesh with `levels` levels (paper, Algorithm 1;
 * level 0 is the coarsest, N_l = N / 2^(levels-1-l)).  Rediscretises the
 * operator on every level, assembles and inverts (partial-pivot LU, FP64)
 * the 25 distinct Vanka patch matrices of every relaxed level (paper,
 * subsection "Vanka patch matrices": 25 patch matrices on a uniform mesh,
 * independent of N), and the bordered coarsest-level matrix.  Allocates the
 * device workspace on the current HIP device; `hip_stream` is used for the
 * uploads and is synchronised before return.
 * Requirements: nx == ny; levels >= 2; nx divisible by 2^(levels-1);
 * coarsest mesh at least 2 x 2; nu > 0 and finite; opts NULL or with
 * nu_pre, nu_post in [0, 16], 0 < omega <= 2, batch in [1, 64].  Violations give
 * VKMG_ERR_INVALID_ARG; a singular patch gives VKMG_ERR_SINGULAR_PATCH.
 */
vkmg_status vkmg_setup(const vkmg_grid* grid, int32_t levels, double nu,
                       const vkmg_options* opts, void* hip_stream, vkmg_ctx** out);

/*
 * As vkmg_setup for a per-element viscosity (paper, bilinear form a(u,v) =
 * nu (grad u, grad v) with nu constant on each element; the extension to
 * variable coefficients for which the paper notes that the shared-inverse
 * Vanka does not apply): nu_elem holds nx*nx positive values on the host,
 * element (ex, ey) at index ey*nx + ex.  Coarser levels take the
 * arithmetic mean of the four children.  Every Vanka patch then has its own
 * inverse ("simple" Vanka: (N_l+1)^2 x 51 x 51 stored weighted inverses per
 * relaxed level, formed on the host threads); the residual sums the element
 * matrices scaled by nu_e.  Requires Vanka relaxation (VKMG_ERR_UNSUPPORTED
 * otherwise); interior_apply is ignored.  Errors as vkmg_setup.
 */
vkmg_status vkmg_setup_viscosity(const vkmg_grid* grid, int32_t levels, const double* nu_elem,
                                 const vkmg_options* opts, void* hip_stream, vkmg_ctx** out);

/* Destroy a context (NULL-safe).  Waits for the device to finish its work. */
void vkmg_destroy(vkmg_ctx* ctx);

/* Sizes and offsets of the finest level (level = levels-1) or of `level`. */
vkmg_status vkmg_layout_of(const vkmg_ctx* ctx, vkmg_layout* out);
vkmg_status vkmg_level_layout(const vkmg_ctx* ctx, int32_t level, vkmg_layout* out);
vkmg_status vkmg_num_levels(const vkmg_ctx* ctx, int32_t* out);

/*
 * r = b - A x on the finest level, FP64 (the residual of Algorithm 1 and of
 * FGMRES).  b, x, r: n doubles each; r must not alias x.  A is applied
 * matrix-free: Dirichlet entries of x are treated as zero columns and the
 * Dirichlet rows return b - x.
 */
vkmg_status vkmg_residual(vkmg_ctx* ctx, const double* b, const double* x, double* r, void* stream);

/* y = A x on the finest level, FP64 (same conventions). */
vkmg_status vkmg_apply(vkmg_ctx* ctx, const double* x, double* y, void* stream);

/*
 * Right-hand side of the constrained system on the finest level:
 *   b_F = (M f)_F - A_FD g,  b_D = g_D,  b_p = -B_pD g
 * where M is the Q2 mass matrix (so M f is the load of the body force whose
 * Q2 interpolant has nodal values f) and g holds the Dirichlet data.
 * f, g: 2*(2N+1)^2 doubles each ([f_x | f_y], only the boundary entries of
 * g are read; g may be NULL for homogeneous data); b: n doubles, FP64.
 * Contexts with a per-element viscosity take g == NULL only
 * (VKMG_ERR_UNSUPPORTED otherwise).
 */
vkmg_status vkmg_assemble_rhs(vkmg_ctx* ctx, const double* f, const double* g, double* b,
                              void* stream);

/*
 * Transpose of the force-to-load map of vkmg_assemble_rhs (the part
 * f -> (M f)_F of b; for the adjoint of a solve with respect to the body
 * force): grad_f = M^T R_F^T lam, i.e. grad_f(k) = sum over the free
 * velocity DoFs i of M_ik lam_u(i), per component.  lam: n doubles (only its
 * velocity block on free nodes is read); grad_f: 2 (2N+1)^2 doubles, FP64,
 * finest level.  Asynchronous.
 */
vkmg_status vkmg_assemble_rhs_adjoint(vkmg_ctx* ctx, const double* lam, double* grad_f,
                                      void* stream);

/*
 * Gradient of a loss with respect to a per-element viscosity, from the
 * adjoint state lam (A lam = P dL/dx) and the solution x: grad_nu[e] =
 * -sum over both velocity components of lam_e^T L_e x_e on the free nodes
 * of element e (L_e the Q2 element Laplacian per unit viscosity; the
 * derivative of A with respect to nu_e).  lam, x: n doubles; grad_nu: nx*nx
 * doubles (index ey*nx + ex); FP64, finest level.  Asynchronous.
 */
vkmg_status vkmg_viscosity_gradient(vkmg_ctx* ctx, const double* lam, const double* x,
                                    double* grad_nu, void* stream);

/*
 * x_p -= mean(x_p): removes the constant-pressure null-space component of an
 * FP64 finest-level vector (plain mean over the (N+1)^2 pressure DoFs; an
 * orthogonal projection, so it is its own adjoint).  Asynchronous.
 */
vkmg_status vkmg_remove_pressure_mean(vkmg_ctx* ctx, double* x, void* stream);

/*
 * Dirichlet lifting of an FP64 finest-level vector: x = b on the Dirichlet
 * DoFs (both velocity components at every boundary Q2 node; paper, section
 * "Problem setup": Dirichlet velocity on every edge), x = 0 on every other
 * DoF.  Since the Dirichlet rows of the constrained system are identity
 * rows with b_D = g_D, lifting the right-hand side gives the initial guess
 * that vkmg_fgmres_solve expects (and, for an adjoint system A lam = r,
 * the exact values of lam on the decoupled Dirichlet rows).  b, x: n
 * doubles (B vectors in a batched context); x may alias b.  Asynchronous.
 */
vkmg_status vkmg_dirichlet_lift(vkmg_ctx* ctx, const double* b, double* x, void* stream);

/*
 * One additive Vanka sweep on `level` (1 <= level <= levels-1), in the
 * context's multigrid precision (x, b are double for VKMG_FP64 contexts and
 * float for VKMG_FP32 contexts): r = b - A_l x, then
 * x += sum_i V_i^T W_i A_i^{-1} V_i r over all patches i (paper, equation
 * "vksystem" and Algorithm 3), W_i = omega diag(1/m_j) with m_j the number
 * of patches containing DoF j and zero weight on Dirichlet DoFs.  x is
 * updated in place; b is read-only and must not alias x.
 */
vkmg_status vkmg_vanka_sweep(vkmg_ctx* ctx, int32_t level, void* x, const void* b, void* stream);

/*
 * The update half of a sweep, given the residual: x += sum_i V_i^T W_i
 * A_i^{-1} V_i r (patch gather, patch-inverse apply and weighted scatter of
 * Algorithm 3, without forming r).  Same level range, precision and
 * operator as vkmg_vanka_sweep; r is read-only and must not alias x; r
 * must vanish on Dirichlet DoFs for the result to equal a sweep (their
 * weights are zero, so they are never read into a correction).
 */
vkmg_status vkmg_vanka_update(vkmg_ctx* ctx, int32_t level, void* x, const void* r, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * update as vkmg_vanka_update, with the same arguments and results (the
 * same kernels), except that the patch corrections the update keeps
 * between its two launches live in a static device array of the library
 * (4 MiB per GPU, held until the process ends) instead of the context's
 * buffer.  Calls no hipMalloc, hipFree or other allocating routine.
 * Limit: the corrections must fit, i.e. 64 * (8N - 8) values of the
 * multigrid precision per right-hand side for a level of N elements per
 * side (N <= 1024 in FP64, N <= 2048 in FP32, for one right-hand side), or
 * 64 * (N + 1)^2 per right-hand side for a per-element viscosity; larger
 * levels or batches return VKMG_ERR_INVALID_ARG before any launch.  Every
 * call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other streams, other contexts, other host threads) race and
 * must be serialised by the caller.  Nothing in the array needs to start
 * at zero (each update writes every value it reads).
 */
vkmg_status vkmg_vanka_update_noalloc(vkmg_ctx* ctx, int32_t level, void* x, const void* r,
                                      void* stream);

/*
 * One sweep of the context's relaxation (opts.relaxation) on `level`
 * (1 <= level <= levels-1), in the multigrid precision: r = b - A_l x, then
 * the Vanka update (as vkmg_vanka_sweep) or the Braess-Sarazin update
 * (paper, Algorithm 2 with the equations bseq1/bseq2; see
 * vkmg_relaxation).  x is updated in place; b must not alias x.
 */
vkmg_status vkmg_relax(vkmg_ctx* ctx, int32_t level, void* x, const void* b, void* stream);

/*
 * Grid transfers of Algorithm 1 in the multigrid precision:
 *   vkmg_restrict:   b_coarse = P^T r_fine   (fine = level, coarse = level-1)
 *   vkmg_prolong_add: x_fine += P e_coarse
 * P is the finite-element interpolation from the level-1 Q2/Q1 spaces to
 * the level ones, with rows of fine Dirichlet DoFs and columns of coarse
 * Dirichlet DoFs zeroed.  1 <= level <= levels-1.
 */
vkmg_status vkmg_restrict(vkmg_ctx* ctx, int32_t level, const void* r_fine, void* b_coarse,
                          void* stream);
vkmg_status vkmg_prolong_add(vkmg_ctx* ctx, int32_t level, const void* e_coarse, void* x_fine,
                             void* stream);

/*
 * Exact coarsest-level solve e = A_0^+ r (Algorithm 1, level 0), through the
 * precomputed inverse of the matrix bordered by the constant-pressure
 * vector, computed in FP64; r and e in the multigrid precision, n_0 values.
 */
vkmg_status vkmg_coarse_solve(vkmg_ctx* ctx, const void* r, void* e, void* stream);

/*
 * One multigrid V(nu_pre, nu_post) cycle with zero initial guess on every
 * level (Algorithm 1): z = M r.  r, z: n doubles on the finest level (the
 * V-cycle itself runs in the context's multigrid precision; FP32 contexts
 * round r to float on entry and widen z on exit).  z must not alias r.
 */
vkmg_status vkmg_vcycle(vkmg_ctx* ctx, const double* r, double* z, void* stream);

/*
 * Launch shapes of the V-cycle, per level size.  No choice changes a
 * result: every alternative does the same arithmetic in the same order, so
 * V-cycles and solves are bitwise the same under any tuning.
 *   fused_sweep_max_n:   levels with 16 <= N <= this run each Vanka sweep
 *                        of a V-cycle as one launch (residual, boundary
 *                        patches, interior patches and owner sums of one
 *                        tile in one workgroup) instead of three; 0: never.
 *                        Vanka contexts with constant viscosity, vector
 *                        apply and nu_pre, nu_post >= 1 only.
 *   park_min_n:          FP64 levels with N >= this use the tile kernel that
 *                        parks half of a patch in LDS during the interior
 *                        apply (three waves per SIMD instead of two).
 *   fused_prolong_max_n: FP64 levels with N <= this add the coarse-grid
 *                        correction inside the residual launch of the first
 *                        post-smoothing sweep (FP32 contexts: every level).
 *   boundary_per_wave:   boundary patches per wavefront in the boundary-
 *                        patch launch: 1, 2, 4 or 8; 0: from the patch count.
 * Defaults are the choices measured fastest on MI355X for the context's
 * precision (vkmg_setup); vkmg_autotune measures them on the running GPU.
 */
typedef struct {
    int32_t fused_sweep_max_n;
    int32_t park_min_n;
    int32_t fused_prolong_max_n;
    int32_t boundary_per_wave;
} vkmg_tuning;

vkmg_status vkmg_get_tuning(const vkmg_ctx* ctx, vkmg_tuning* out);
/* Invalid values (negative sizes, boundary_per_wave not 0/1/2/4/8) return
 * VKMG_ERR_INVALID_ARG and leave the tuning unchanged. */
vkmg_status vkmg_set_tuning(vkmg_ctx* ctx, const vkmg_tuning* tuning);

/*
 * Measure the tuning on this GPU: coordinate descent over the four fields
 * (candidates: the context's level sizes), two rounds, each candidate timed
 * as the median of three runs of `reps` V-cycles (reps >= 1) replayed from a
 * captured graph on `stream`, with the context's own work vectors as input
 * (overwritten); a candidate replaces the current choice only if it is more
 * than 1 % faster.  The result becomes the context's tuning and, if `out`
 * is not NULL, is copied there.  Synchronises `stream`; allocates events and
 * graphs, frees them before returning.
 */
vkmg_status vkmg_autotune(vkmg_ctx* ctx, int32_t reps, void* stream, vkmg_tuning* out);

/*
 * Solve A x = b by restarted flexible GMRES right-preconditioned with
 * vkmg_vcycle (paper, section "Overall solver performance"), in FP64.
 * x holds the initial guess on entry (use the Dirichlet lifting: g on D,
 * zero elsewhere) and the solution on exit.  Stops when the rotated
 * residual estimate and then the recomputed residual satisfy
 * ||b - A x|| <= rtol ||b - A x0||; restarts every `restart` steps
 * (1..256); at most max_iters Arnoldi steps (>= 1).  Returns VKMG_OK,
 * VKMG_ERR_NOT_CONVERGED (x is the last iterate: max_iters reached, or a
 * restart cycle whose estimate met rtol left the recomputed residual above
 * it and not halved, i.e. rtol is below the rounding floor of the system)
 * or VKMG_ERR_NONFINITE; `info` (may be NULL) is filled in every case.
 * Batched contexts (batch B > 1) solve the B systems independently (own
 * Krylov bases, rotations, stopping tests and restarts; one batched launch
 * per kernel for all of them, steps of right-hand sides that have already
 * converged are computed and discarded); `info` then points to B entries,
 * max_iters bounds the Arnoldi steps of each, restart must be <= 32
 * (VKMG_ERR_UNSUPPORTED otherwise), and the return value is VKMG_OK if all
 * B converged, else the status of the first that did not.
 */
vkmg_status vkmg_fgmres_solve(vkmg_ctx* ctx, const double* b, double* x, double rtol,
                              int32_t restart, int32_t max_iters, vkmg_info* info, void* stream);

/*
 * Per-kernel device timing.  While bit k of `class_mask` is set, the
 * library brackets every launch of kernel class k (vkmg_kernel_class) with
 * a pair of HIP events recorded on the launch stream, tagged with the
 * multigrid level it ran on (-1 for the FGMRES vector kernels).  A Vanka
 * "launch" is the update of one sweep (the interior-tile and boundary-tile
 * kernels together).  vkmg_set_timing discards all previous records;
 * mask 0 stops recording.  vkmg_kernel_timing waits for the recorded events
 * and returns, for class `kernel_class` and level `level` (-1 = all
 * levels), the number of bracketed launches and their summed duration in
 * milliseconds.  Records accumulate until the next vkmg_set_timing.
 */
vkmg_status vkmg_set_timing(vkmg_ctx* ctx, int32_t class_mask);
vkmg_status vkmg_kernel_timing(vkmg_ctx* ctx, int32_t kernel_class, int32_t level,
                               int64_t* launches, double* total_ms);

/*
 * Host-only (no GPU needed): the Vanka patch matrix A_i = V_i A V_i^T of
 * patch class `cls` (0..24, cls = 5*class_y + class_x, class 0 = on the low
 * boundary, 1 = one element in, 2 = interior, 3 = one element from the high
 * boundary, 4 = on the high boundary) on an N x N mesh (N >= 4) with
 * viscosity nu, in the 51-slot patch numbering: u_x at the 5x5 Q2 nodes
 * (2I-2+a, 2J-2+b) in slot 5b+a, u_y in slot 25+5b+a, the pressure in slot
 * 50.  Absent slots (outside the domain) get an identity row and column and
 * present[s] = 0.  Outputs (caller-owned host memory): A (51*51, row-major),
 * Ainv (51*51, its inverse), Wainv (51*51, the weighted inverse
 * W A^{-1} with omega = `omega`, zero rows on Dirichlet and absent slots),
 * present (51).  Any output may be NULL.
 */
vkmg_status vkmg_host_patch_matrix(int32_t N, double nu, double omega, int32_t cls, double* A,
                                   double* Ainv, double* Wainv, uint8_t* present);

const char* vkmg_status_string(vkmg_status s);
const char* vkmg_last_error(void); /* thread-local; "" if none */

#ifdef __cplusplus
}
#endif

#endif /* VKMG_H */
