// Launchers of the vkmg HIP kernels (kernels.hip).  All launches are
// asynchronous on `stream`; shapes are validated by the callers.
#pragma once

#include <hip/hip_runtime.h>

#include "vkmg_internal.h"

namespace vkmg {

// r = b - A x (mode 0) or r = A x (mode 1, b unused); Ti: type of x,
// To: type of b and r, arithmetic in To.
template <typename Tx, typename T>
void launch_residual(const Geom& g, const T* b, const Tx* x, T* r, int mode, hipStream_t s);

// b = M f - A_FD g on free rows, g on Dirichlet rows, -B_pD g on pressure rows.
void launch_rhs(const Geom& g, const double* f, const double* gd, double* b, hipStream_t s);

// One Vanka update given the residual r of x_in:
// x_out = x_in + sum_i V_i^T W_i A_i^{-1} V_i r (x_out == x_in allowed;
// x_in == nullptr means x_in = 0, so r = b).  `table` is the level's
// patch-operator table (kLevelTable values: the 25 weighted inverses stored
// transposed, then the interior reflection blocks, which the kernels take
// from compile-time constants instead); `dbuf` is scratch for the boundary
// patches (vanka_boundary_scratch(N) values).  The interior patches are
// applied on the matrix instructions with the operand table `mtab`
// (kMfmaTable values, mfma_interior_table) when `mfma`, else on the vector
// ALUs with the compile-time constants.
template <typename T>
void launch_vanka_update(const Geom& g, const T* r, const T* xin, T* xout, const T* table,
                         const T* mtab, T* dbuf, double omega, bool mfma, hipStream_t s);
int64_t vanka_boundary_scratch(int N);

// Transfers between the fine level gf and the coarse level gc (gf.N == 2 gc.N).
template <typename T>
void launch_restrict(const Geom& gf, const Geom& gc, const T* rf, T* bc, hipStream_t s);
template <typename T>
void launch_prolong_add(const Geom& gf, const Geom& gc, const T* ec, T* xf, hipStream_t s);

// e = C r with C (n x n, FP64) the coarse bordered inverse.
template <typename T>
void launch_coarse_gemv(int64_t n, const double* C, const T* r, T* e, hipStream_t s);

// Elementwise helpers.
template <typename T>
void launch_fill_zero(T* x, int64_t n, hipStream_t s);
template <typename Ti, typename To>
void launch_cast(const Ti* in, To* out, int64_t n, hipStream_t s);

// Krylov kernels (FP64).  V: k vectors of length n with stride ldv.
constexpr int kDotBlocks = 2048;
// part[v * kDotBlocks + blk] = partial dot of V_v and w
void launch_mdot_partial(const double* V, int64_t ldv, int k, const double* w, int64_t n,
                         double* part, hipStream_t s);
// out[v] = sum of the kDotBlocks partials of vector v (k vectors)
void launch_reduce_partials(const double* part, int k, double* out, hipStream_t s);
// w -= sum_v h[v] V_v
void launch_update(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t n,
                   hipStream_t s);
// w -= sum_v h[v] V_v, then partials of V^T w (k values) and ||w||^2 (one
// more) into part; k <= 32
void launch_update_dot(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t n,
                       double* part, hipStream_t s);
// out = (w - V h2) / sqrt(nrm2[0] - |h2|^2); k <= 32
void launch_normalize(const double* V, int64_t ldv, int k, const double* h2, const double* nrm2,
                      const double* w, double* out, int64_t n, hipStream_t s);
// Delayed CGS2, pass 1 (j < 32 final vectors V, unnormalised u, w):
// partials of V^T w (j rows), V^T u (j rows), u.u, u.w, w.w into part
void launch_dcgs_dots(const double* V, int64_t ldv, int j, const double* u, const double* w,
                      int64_t n, double* part, hipStream_t s);
// Delayed CGS2, pass 2 from the 2j+3 reduced values c: u <- v_j (final),
// next <- normalised successor; cf = (alpha, gamma, d, 1/sqrt(d))
void launch_dcgs_update(const double* V, int64_t ldv, int j, const double* c, double* u,
                        const double* w, double* next, int64_t n, double* cf, hipStream_t s);
// x += sum_v y[v] Z_v
void launch_axpy_multi(const double* Z, int64_t ldz, int k, const double* y, double* x, int64_t n,
                       hipStream_t s);
// out = alpha * in
void launch_scale(const double* in, double alpha, double* out, int64_t n, hipStream_t s);

}  // namespace vkmg
