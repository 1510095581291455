// Launchers of the vkmg HIP kernels (kernels.hip).  All launches are
// asynchronous on `stream`; shapes are validated by the callers.
//
// Batches: launchers taking `nb` process nb right-hand sides in one launch
// (a grid dimension of the kernel).  The vectors of a batch lie back to back
// in memory, n of their level apart (n = 2 (2N+1)^2 + (N+1)^2), and the
// boundary-patch scratch of launch_vanka_update holds nb blocks of
// vanka_boundary_scratch(N) values.
#pragma once

#include <hip/hip_runtime.h>

#include "vkmg_internal.h"

namespace vkmg {

// r = b - A x (mode 0) or r = A x (mode 1, b unused); Ti: type of x,
// To: type of b and r, arithmetic in To.
// nue: per-element viscosity (N^2 values, index ey*N + ex) or nullptr for
// the constant g.nu.
template <typename Tx, typename T>
void launch_residual(const Geom& g, const T* b, const Tx* x, T* r, int mode, hipStream_t s,
                     int nb = 1, const T* nue = nullptr);

// y = A x (FP64 operator, as launch_residual mode 1) for an FP32 x, which is
// also written widened to FP64 into x64.
void launch_apply_widen(const Geom& g, const float* x, double* y, double* x64, hipStream_t s,
                        const double* nue = nullptr, int nb = 1);

// x2 = x + P ec (the prolongation of the coarse correction ec, as
// launch_prolong_add) and r = b - A x2 in one pass over the fine level g
// (coarse level gc); x is not modified.  nue as for launch_residual.
template <typename T>
void launch_residual_prolong(const Geom& g, const Geom& gc, const T* b, const T* x, const T* ec,
                             T* x2, T* r, hipStream_t s, int nb = 1, const T* nue = nullptr);

// b = M f - A_FD g on free rows, g on Dirichlet rows, -B_pD g on pressure
// rows (f, g: 2 (2N+1)^2 values per right-hand side).
void launch_rhs(const Geom& g, const double* f, const double* gd, double* b, hipStream_t s,
                int nb = 1);

// grad_f = transpose of f -> (M f)_F (the force part of launch_rhs) applied
// to lam (n values per right-hand side; its velocity block is read on free
// nodes); grad_f: 2 (2N+1)^2 values per right-hand side.
void launch_rhs_adjoint(const Geom& g, const double* lam, double* grad, hipStream_t s, int nb = 1);
// grad[e] = -sum_c lam_{c,e}^T L_e x_{c,e} over the free Q2 nodes of element e
// (N^2 values per right-hand side, index ey*N + ex).
void launch_visc_grad(const Geom& g, const double* lam, const double* x, double* grad,
                      hipStream_t s, int nb = 1);
// x_p -= mean(x_p) on every right-hand side (FP64): partial sums in part
// (256 per entry), the sums at sums[entry * so].
void launch_pressure_mean_zero(const Geom& g, double* x, double* part, double* sums, int64_t so,
                               hipStream_t s, int nb = 1);

// One Vanka update given the residual r of x_in:
// x_out = x_in + sum_i V_i^T W_i A_i^{-1} V_i r (x_out == x_in allowed;
// x_in == nullptr means x_in = 0, so r = b).  `table` is the level's
// patch-operator table (kLevelTable values: the 25 weighted inverses stored
// transposed, then the interior reflection blocks, which the kernels take
// from compile-time constants instead); `dbuf` is scratch for the boundary
// patches (vanka_boundary_scratch(N) values per right-hand side).  The
// interior patches are applied on the matrix instructions with the operand
// table `mtab` (kMfmaTable values, mfma_interior_table) when `mfma`, else on
// the vector ALUs with the compile-time constants.  Launch shape only (the
// results do not depend on them): `park` selects the FP64 tile kernel that
// parks half of a patch in LDS during the apply (160 instead of 229 VGPRs,
// three waves per SIMD instead of two); `per_wave` boundary patches per
// wavefront (1, 2, 4 or 8; 0: from the patch count).
template <typename T>
void launch_vanka_update(const Geom& g, const T* r, const T* xin, T* xout, const T* table,
                         const T* mtab, T* dbuf, double omega, bool mfma, hipStream_t s,
                         int nb = 1, bool park = false, int per_wave = 0);
// The two launches of launch_vanka_update, in that order: the boundary-patch
// corrections into dbuf, then the interior tiles (which also commit dbuf).
template <typename T>
void launch_vanka_boundary(const Geom& g, const T* r, const T* table, T* dbuf, hipStream_t s,
                           int nb = 1, int per_wave = 0);
template <typename T>
void launch_vanka_tiles(const Geom& g, const T* r, const T* xin, T* xout, const T* mtab,
                        const T* dbuf, double omega, bool mfma, hipStream_t s, int nb = 1,
                        bool park = false);
int64_t vanka_boundary_scratch(int N);
// One complete Vanka sweep in one launch (levels with N >= vanka_fused_min_n()):
// r = b - A x_in and x_out = x_in + sum_i V_i^T W_i A_i^{-1} V_i r, bitwise
// the residual launch followed by launch_vanka_update (vector apply).
// x_out must not alias x_in; x_in == nullptr means x_in = 0 (r = b).
// `table` as for launch_vanka_update.  No scratch.
template <typename T>
void launch_vanka_fused(const Geom& g, const T* b, const T* xin, T* xout, const T* table,
                        double omega, hipStream_t s, int nb = 1);
int vanka_fused_min_n();
// Vanka update with one stored weighted inverse per patch ("simple" Vanka,
// for a per-element viscosity): `tables` holds (N+1)^2 transposed 51 x 51
// inverses (simple_vanka_tables), `dbuf` (N+1)^2 * 64 values per
// right-hand side.
template <typename T>
void launch_vanka_simple(const Geom& g, const T* r, const T* xin, T* xout, const T* tables,
                         T* dbuf, hipStream_t s, int nb = 1);

// One Braess-Sarazin relaxation (inexact form) given the residual r of x_in
// (x_in == nullptr: x_in = 0, r = b): rhs = r_p - (1/t) B D^{-1} r_u into
// prhs, `jacobi_sweeps` weighted-Jacobi sweeps on S dp = rhs from dp = 0
// (S = -(1/t) B D^{-1} B^T, scratch vtmp of 2 (2N+1)^2 values), then
// x_out = x_in + omega [ (1/t) D^{-1} (r_u - B^T dp); dp ].  prhs and dp hold
// (N+1)^2 values per right-hand side.
template <typename T>
void launch_bs_relax(const Geom& g, const T* r, const T* xin, T* xout, T* prhs, T* dp, T* vtmp,
                     double t, double omega, double jacobi_weight, int jacobi_sweeps,
                     hipStream_t s, int nb = 1);

// Transfers between the fine level gf and the coarse level gc (gf.N == 2 gc.N).
template <typename T>
void launch_restrict(const Geom& gf, const Geom& gc, const T* rf, T* bc, hipStream_t s,
                     int nb = 1);
template <typename T>
void launch_prolong_add(const Geom& gf, const Geom& gc, const T* ec, T* xf, hipStream_t s,
                        int nb = 1);

// e = C r with C (n x n, FP64) the coarse bordered inverse.
template <typename T>
void launch_coarse_gemv(int64_t n, const double* C, const T* r, T* e, hipStream_t s, int nb = 1);

// Elementwise helpers (n values in total).
template <typename T>
void launch_fill_zero(T* x, int64_t n, hipStream_t s);
template <typename Ti, typename To>
void launch_cast(const Ti* in, To* out, int64_t n, hipStream_t s);
// x = b on the Dirichlet DoFs of level g, 0 elsewhere (nb vectors, FP64).
void launch_lift(const Geom& g, const double* b, double* x, hipStream_t s, int nb = 1);

// Per-system area of the device-side FGMRES of the delayed scheme
// (restart <= kMaxRestart), `stride` doubles apart (offsets in doubles):
// the reduced dots of a step, its pass-2 coefficients, the solution of the
// small system, the pressure-mean scratch, then the Givens state.  The
// scalars are doubles (flags 0/1, counts exact).
struct GivensLayout {
    static constexpr int kMaxRestart = 32;
    static constexpr int kDots = 0;       // 2j + 3 reduced values of pass 1
    static constexpr int kCoef = 300;     // alpha, gamma, d, sigma of pass 2
    static constexpr int kY = 600;        // y (kMaxRestart)
    static constexpr int kScale = 900;    // 1 / beta at the start of a cycle
    static constexpr int kMean = 1000;    // pressure-mean scratch
    static constexpr int kCs = 1100;      // cos of the rotations (kMaxRestart)
    static constexpr int kSn = 1140;      // sin
    static constexpr int kGbase = 1180;   // rhs after the final rotations (kMaxRestart + 1)
    static constexpr int kGv = 1220;      // rhs after the provisional rotation too
    static constexpr int kHcol = 34;      // one unrotated Hessenberg column
    static constexpr int kHcols = 1260;   // two of them (step parity)
    static constexpr int kR = 1330;       // rotated columns, column j at j(j+3)/2, j+2 values
    static constexpr int kScalars = 1900;
    // scalar slots (kScalars + ...)
    static constexpr int kBeta0 = 0, kTarget = 1, kBeta = 2, kSigmaPrev = 3, kEst = 4,
                         kActive = 5, kIters = 6, kKdone = 7, kStatus = 8, kMaxIters = 9,
                         kCycled = 10, kNumScalars = 11;
    static constexpr int kSize = 1920;
};
static_assert(GivensLayout::kR + 32 * 35 / 2 <= GivensLayout::kScalars, "packed R fits");

// Start of a restart cycle for nsys systems (areas `stride` apart): init
// holds 8 values per system (beta0, target, beta, estimate, active flag,
// iterations so far, iteration limit, 1/beta); the Givens state is reset
// and stat (8 values per system: estimate, active, iterations, kdone,
// status, |g_kdone|, cycled) initialised.  The Givens steps themselves run
// inside launch_dcgs_update.
void launch_givens_init(double* area, int64_t stride, const double* init, double* stat, int nsys,
                        hipStream_t s);
// y of every system from its rotated system (zeros from kdone to kmax).
void launch_givens_solve(double* area, int64_t stride, int kmax, int nsys, hipStream_t s);

// Krylov kernels (FP64).  V: k vectors of length n with stride ldv; with
// nb > 1 the batch entries of every vector are sb apart.  Partial sums:
// dot_blocks(nb) = kDotBlocks per row and batch entry (the same partition
// for every batch size).
constexpr int kDotBlocks = 2048;
int dot_blocks(int nb);
// part[(b * k + v) * G + blk] = partial dot of V_v and w of batch entry b
// (G = dot_blocks(nb); k > 32 only for nb == 1)
void launch_mdot_partial(const double* V, int64_t ldv, int k, const double* w, int64_t n,
                         double* part, hipStream_t s, int nb = 1, int64_t sb = 0);
// out[b * so + v] = sum of the G partials of row v of batch entry b
void launch_reduce_partials(const double* part, int k, double* out, hipStream_t s, int nb = 1,
                            int64_t so = 0);
// w -= sum_v h[v] V_v (single right-hand side)
void launch_update(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t n,
                   hipStream_t s);
// w -= sum_v h[v] V_v, then partials of V^T w (k values) and ||w||^2 (one
// more) into part; k <= 32, single right-hand side
void launch_update_dot(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t n,
                       double* part, hipStream_t s);
// out = (w - V h2) / sqrt(nrm2[0] - |h2|^2); k <= 32, single right-hand side
void launch_normalize(const double* V, int64_t ldv, int k, const double* h2, const double* nrm2,
                      const double* w, double* out, int64_t n, hipStream_t s);
// Delayed CGS2, pass 1 (j < 32 final vectors V, unnormalised u, w):
// partials of V^T w (j rows), V^T u (j rows), u.u, u.w, w.w into part
// (2j+3 rows per batch entry)
void launch_dcgs_dots(const double* V, int64_t ldv, int j, const double* u, const double* w,
                      int64_t n, double* part, hipStream_t s, int nb = 1, int64_t sb = 0);
// Delayed CGS2, pass 2 from the 2j+3 reduced values c: u <- v_j (final),
// next <- normalised successor; cf = (alpha, gamma, d, 1/sqrt(d)); c and cf
// of batch entry b at offset b * sc.  next32: if given, also next rounded
// to FP32 (the input of an FP32 V-cycle), vectors sb apart.
// With garea (GivensLayout areas sc apart, cf inside them), block 0 of
// every batch entry also runs the entry's Givens step (summary to
// gstat[8 * entry ...], see launch_givens_init).
void launch_dcgs_update(const double* V, int64_t ldv, int j, const double* c, double* u,
                        const double* w, double* next, int64_t n, double* cf, hipStream_t s,
                        int nb = 1, int64_t sb = 0, int64_t sc = 0, float* next32 = nullptr,
                        double* garea = nullptr, double* gstat = nullptr);
// x += sum_v y[v] Z_v; y of batch entry b at offset b * sy
void launch_axpy_multi(const double* Z, int64_t ldz, int k, const double* y, double* x, int64_t n,
                       hipStream_t s, int nb = 1, int64_t sb = 0, int64_t sy = 0);
// out = alpha * in
void launch_scale(const double* in, double alpha, double* out, int64_t n, hipStream_t s);
// out_b = alpha[b * sa] * in_b, in_b at in + b * sin, out_b at out + b * sout
void launch_scale_batched(const double* in, int64_t sin, const double* alpha, int64_t sa,
                          double* out, int64_t sout, int64_t n, int nb, hipStream_t s);

}  // namespace vkmg
