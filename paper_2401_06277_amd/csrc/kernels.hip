// HIP kernels of the vkmg library for gfx950 (CDNA4, wave64).
//
// Layout of every level vector: [u_x | u_y | p], Q2 blocks of (2N+1)^2 and a
// Q1 block of (N+1)^2 values, row-major (index j*side + i).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "stencil.h"

namespace vkmg {

namespace {

__device__ __forceinline__ bool q2_boundary(int qi, int qj, int s2) {
    return qi == 0 || qj == 0 || qi == s2 - 1 || qj == s2 - 1;
}

// Velocity value with Dirichlet (boundary) columns read as zero.  Callers
// guarantee 0 <= qi, qj < s2.
template <typename Tx>
__device__ __forceinline__ Tx ld_free(const Tx* __restrict__ u, int qi, int qj, int s2) {
    return q2_boundary(qi, qj, s2) ? Tx(0) : u[int64_t(qj) * s2 + qi];
}

// ---------------------------------------------------------------------------
// Operator rows
// ---------------------------------------------------------------------------

// (A x) at the free Q2 node (i,j) of parity (PX, PY), both components.
template <int PX, int PY, typename Tx, typename T>
__device__ __forceinline__ void velocity_rows(const Geom& g, const Tx* __restrict__ ux,
                                              const Tx* __restrict__ uy,
                                              const Tx* __restrict__ p, int i, int j, T& ax,
                                              T& ay) {
    T lx = 0, ly = 0;
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy) {
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            const int c = st_L(PY, PX, dy, dx);
            if (c != 0) {
                lx += T(c) * T(ld_free(ux, i + dx, j + dy, g.s2));
                ly += T(c) * T(ld_free(uy, i + dx, j + dy, g.s2));
            }
        }
    }
    T bx = 0, by = 0;
#pragma unroll
    for (int oy = -2; oy <= 2; ++oy) {
        if (((oy - PY) & 1) != 0) continue;
#pragma unroll
        for (int ox = -2; ox <= 2; ++ox) {
            if (((ox - PX) & 1) != 0) continue;
            const int cx = st_Mq(oy) * st_G(ox);
            const int cy = st_G(oy) * st_Mq(ox);
            if (cx == 0 && cy == 0) continue;
            const int I = (i - ox) / 2, J = (j - oy) / 2;
            const T pv = T(p[int64_t(J) * g.s1 + I]);
            bx += T(cx) * pv;
            by += T(cy) * pv;
        }
    }
    const T cl = T(g.nu / 90.0), cb = T(-g.h / 36.0);
    ax = cl * lx + cb * bx;
    ay = cl * ly + cb * by;
}

// (B u) at the Q1 node (I,J).
template <typename Tx, typename T>
__device__ __forceinline__ T pressure_row(const Geom& g, const Tx* __restrict__ ux,
                                          const Tx* __restrict__ uy, int I, int J) {
    T s = 0;
#pragma unroll
    for (int oy = -2; oy <= 2; ++oy) {
#pragma unroll
        for (int ox = -2; ox <= 2; ++ox) {
            const int cx = st_Mq(oy) * st_G(ox);
            const int cy = st_G(oy) * st_Mq(ox);
            if (cx == 0 && cy == 0) continue;
            const int qi = 2 * I + ox, qj = 2 * J + oy;
            if (qi < 1 || qj < 1 || qi > g.s2 - 2 || qj > g.s2 - 2) continue;
            const int64_t q = int64_t(qj) * g.s2 + qi;
            s += T(cx) * T(ux[q]) + T(cy) * T(uy[q]);
        }
    }
    return T(-g.h / 36.0) * s;
}

// ---------------------------------------------------------------------------
// Residual r = b - A x (MODE 0) / apply r = A x (MODE 1)
// One thread per cell (ex, ey) in [0,N]^2: Q2 nodes (2ex+a, 2ey+b), a,b in
// {0,1}, and the Q1 node (ex, ey).
// ---------------------------------------------------------------------------

template <int MODE, typename Tx, typename T>
__global__ __launch_bounds__(256) void residual_kernel(Geom g, const T* __restrict__ b,
                                                       const Tx* __restrict__ x,
                                                       T* __restrict__ r) {
    const int ex = blockIdx.x * 16 + (threadIdx.x & 15);
    const int ey = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (ex > g.N || ey > g.N) return;
    const Tx* ux = x;
    const Tx* uy = x + g.nq2;
    const Tx* p = x + 2 * g.nq2;
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) {
            const int i = 2 * ex + aa, j = 2 * ey + bb;
            if (i >= g.s2 || j >= g.s2) continue;
            const int64_t q = int64_t(j) * g.s2 + i;
            T ax, ay;
            if (q2_boundary(i, j, g.s2)) {
                ax = T(ux[q]);
                ay = T(uy[q]);
            } else if (aa == 0 && bb == 0) {
                velocity_rows<0, 0>(g, ux, uy, p, i, j, ax, ay);
            } else if (aa == 1 && bb == 0) {
                velocity_rows<1, 0>(g, ux, uy, p, i, j, ax, ay);
            } else if (aa == 0 && bb == 1) {
                velocity_rows<0, 1>(g, ux, uy, p, i, j, ax, ay);
            } else {
                velocity_rows<1, 1>(g, ux, uy, p, i, j, ax, ay);
            }
            if (MODE == 0) {
                r[q] = b[q] - ax;
                r[g.nq2 + q] = b[g.nq2 + q] - ay;
            } else {
                r[q] = ax;
                r[g.nq2 + q] = ay;
            }
        }
    }
    const int64_t qp = 2 * g.nq2 + int64_t(ey) * g.s1 + ex;
    const T ap = pressure_row<Tx, T>(g, ux, uy, ex, ey);
    r[qp] = (MODE == 0) ? b[qp] - ap : ap;
}

// ---------------------------------------------------------------------------
// Right-hand side: b_F = (M f)_F - (A g_D)_F, b_D = g, b_p = -(B g_D)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double ld_bnd(const double* __restrict__ u, int qi, int qj, int s2) {
    return q2_boundary(qi, qj, s2) ? u[int64_t(qj) * s2 + qi] : 0.0;
}

template <int PX, int PY>
__device__ __forceinline__ void rhs_velocity(const Geom& g, const double* __restrict__ f,
                                             const double* __restrict__ gd, int i, int j,
                                             double& bx, double& by) {
    const double* fx = f;
    const double* fy = f + g.nq2;
    double mx = 0, my = 0, lx = 0, ly = 0;
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy) {
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            const int cm = st_M(PY, dy) * st_M(PX, dx);
            const int64_t q = int64_t(j + dy) * g.s2 + (i + dx);
            if (cm != 0) {
                mx += double(cm) * fx[q];
                my += double(cm) * fy[q];
            }
            const int cl = st_L(PY, PX, dy, dx);
            if (gd != nullptr && cl != 0) {
                lx += double(cl) * ld_bnd(gd, i + dx, j + dy, g.s2);
                ly += double(cl) * ld_bnd(gd + g.nq2, i + dx, j + dy, g.s2);
            }
        }
    }
    const double cmass = g.h * g.h / 900.0, cl = g.nu / 90.0;
    bx = cmass * mx - cl * lx;
    by = cmass * my - cl * ly;
}

__global__ __launch_bounds__(256) void rhs_kernel(Geom g, const double* __restrict__ f,
                                                  const double* __restrict__ gd,
                                                  double* __restrict__ b) {
    const int ex = blockIdx.x * 16 + (threadIdx.x & 15);
    const int ey = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (ex > g.N || ey > g.N) return;
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) {
            const int i = 2 * ex + aa, j = 2 * ey + bb;
            if (i >= g.s2 || j >= g.s2) continue;
            const int64_t q = int64_t(j) * g.s2 + i;
            double bx, by;
            if (q2_boundary(i, j, g.s2)) {
                bx = gd ? gd[q] : 0.0;
                by = gd ? gd[g.nq2 + q] : 0.0;
            } else if (aa == 0 && bb == 0) {
                rhs_velocity<0, 0>(g, f, gd, i, j, bx, by);
            } else if (aa == 1 && bb == 0) {
                rhs_velocity<1, 0>(g, f, gd, i, j, bx, by);
            } else if (aa == 0 && bb == 1) {
                rhs_velocity<0, 1>(g, f, gd, i, j, bx, by);
            } else {
                rhs_velocity<1, 1>(g, f, gd, i, j, bx, by);
            }
            b[q] = bx;
            b[g.nq2 + q] = by;
        }
    }
    double s = 0.0;
    if (gd != nullptr) {
        for (int oy = -2; oy <= 2; ++oy)
            for (int ox = -2; ox <= 2; ++ox) {
                const int qi = 2 * ex + ox, qj = 2 * ey + oy;
                if (qi < 0 || qj < 0 || qi >= g.s2 || qj >= g.s2) continue;
                if (!q2_boundary(qi, qj, g.s2)) continue;
                const int64_t q = int64_t(qj) * g.s2 + qi;
                s += double(st_Mq_row(ey, g.N, oy) * st_G_row(ex, g.N, ox)) * gd[q] +
                     double(st_G_row(ey, g.N, oy) * st_Mq_row(ex, g.N, ox)) * gd[g.nq2 + q];
            }
    }
    // b_p = -(B g_D) with B = -(h/36)(...)
    b[2 * g.nq2 + int64_t(ey) * g.s1 + ex] = (g.h / 36.0) * s;
}

// ---------------------------------------------------------------------------
// Vanka update (owner computes).  A workgroup owns the elements
// [E0, E0+VT) in each direction: the Q2 nodes [2E0, 2E0+2VT) and the Q1
// nodes [E0, E0+VT).  It solves every patch that touches an owned DoF --
// the Q1 nodes [E0-1, E0+VT], VP = VT+2 per direction, one thread each --
// from the residual staged in LDS, and sums the weighted corrections of
// the owned DoFs in a fixed order, so every DoF is written by one
// workgroup and results are bitwise reproducible.
// ---------------------------------------------------------------------------

constexpr int VT = 14;            // owned elements per tile side
constexpr int VP = VT + 2;        // patches per tile side
constexpr int VNT = VP * VP;      // threads per workgroup (256)
constexpr int VR = 2 * VT + 7;    // staged residual region (Q2 nodes per side)
constexpr int VOWN = 2 * VT;      // owned Q2 nodes per side
constexpr int VOWN_PER_THREAD = (VOWN * VOWN + VNT - 1) / VNT;  // 4

// One row of a patch inverse applied to the gathered patch residual.
template <typename T>
__device__ __forceinline__ T row_dot(const T* __restrict__ Mrow, const T (&rv)[kSlots]) {
    T a0 = 0, a1 = 0;
#pragma unroll
    for (int t = 0; t + 1 < kSlots; t += 2) {
        a0 += Mrow[t] * rv[t];
        a1 += Mrow[t + 1] * rv[t + 1];
    }
    a0 += Mrow[kSlots - 1] * rv[kSlots - 1];
    return a0 + a1;
}

__device__ __forceinline__ int dclass(int i, int N) {
    return i == 0 ? 0 : i == N ? 4 : i == 1 ? 1 : i == N - 1 ? 3 : 2;
}

// Tiles whose patches all lie at distance >= 2 from the boundary share the
// interior inverse (INTERIOR = true: the matrix address is a kernel-uniform
// value and is read through the scalar cache); the others (INTERIOR = false,
// launched over all tiles, interior ones returning at once) read the inverse
// of each patch's class per lane.
struct TileRange {
    int lo, hi;  // interior tiles per direction: lo <= t < hi
};

__host__ __device__ inline TileRange interior_tiles(int N) {
    // tile t covers patches [t VT - 1, t VT + VT]; interior class needs
    // 2 <= I <= N - 2
    TileRange r;
    r.lo = 1;
    r.hi = (N - 2 - VT) / VT + 1;  // largest t with t VT + VT <= N - 2, plus one
    if (N - 2 - VT < 0) r.hi = 1;
    if (r.hi < r.lo) r.hi = r.lo;
    return r;
}

template <typename T, bool INTERIOR>
__global__ __launch_bounds__(VNT) void vanka_update_kernel(Geom g, const T* __restrict__ r,
                                                           T* __restrict__ x,
                                                           const T* __restrict__ Wall) {
    __shared__ T s_rx[VR * VR];
    __shared__ T s_ry[VR * VR];
    __shared__ T s_d[VNT * 10];
    const TileRange ir = interior_tiles(g.N);
    int tbx = blockIdx.x, tby = blockIdx.y;
    if (INTERIOR) {
        tbx += ir.lo;
        tby += ir.lo;
    } else if (tbx >= ir.lo && tbx < ir.hi && tby >= ir.lo && tby < ir.hi) {
        return;  // handled by the interior instance
    }
    const int E0x = tbx * VT, E0y = tby * VT;
    const int ox = 2 * E0x - 4, oy = 2 * E0y - 4;
    const int tid = threadIdx.x;
    for (int t = tid; t < VR * VR; t += VNT) {
        const int qi = ox + t % VR, qj = oy + t / VR;
        const bool in = qi >= 0 && qj >= 0 && qi < g.s2 && qj < g.s2;
        const int64_t q = int64_t(qj) * g.s2 + qi;
        s_rx[t] = in ? r[q] : T(0);
        s_ry[t] = in ? r[g.nq2 + q] : T(0);
    }
    const int tx = tid % VP, ty = tid / VP;
    const int I = E0x - 1 + tx, J = E0y - 1 + ty;
    const bool valid = I >= 0 && J >= 0 && I <= g.N && J <= g.N;
    const T rp = valid ? r[2 * g.nq2 + int64_t(J) * g.s1 + I] : T(0);
    __syncthreads();

    T rv[kSlots];
#pragma unroll
    for (int b = 0; b < 5; ++b)
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const int l = (2 * ty + b) * VR + 2 * tx + a;
            rv[5 * b + a] = valid ? s_rx[l] : T(0);
            rv[25 + 5 * b + a] = valid ? s_ry[l] : T(0);
        }
    rv[50] = rp;
    const int cls = INTERIOR ? kInteriorClass
                             : (valid ? 5 * dclass(J, g.N) + dclass(I, g.N) : kInteriorClass);
    const T* __restrict__ M = Wall + cls * kSlots * kSlots;

    T acc_x[VOWN_PER_THREAD], acc_y[VOWN_PER_THREAD];
#pragma unroll
    for (int k = 0; k < VOWN_PER_THREAD; ++k) acc_x[k] = acc_y[k] = T(0);

    // Corrections are produced one patch row (5 nodes, both components) at a
    // time, staged in LDS and pulled by the owners of the DoFs.
#pragma unroll 1
    for (int b = 0; b < 5; ++b) {
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const int sx = 5 * b + a, sy = 25 + 5 * b + a;
            s_d[tid * 10 + a] = row_dot(M + sx * kSlots, rv);
            s_d[tid * 10 + 5 + a] = row_dot(M + sy * kSlots, rv);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < VOWN_PER_THREAD; ++k) {
            const int q = tid + k * VNT;
            if (q >= VOWN * VOWN) continue;
            const int qa = q % VOWN, qb = q / VOWN;
            if (((qb - b) & 1) != 0) continue;
            const int pty = (qb - b) / 2 + 2;
            if (qa & 1) {
#pragma unroll
                for (int a = 1; a < 5; a += 2) {
                    const int ptx = (qa - a) / 2 + 2;
                    acc_x[k] += s_d[(pty * VP + ptx) * 10 + a];
                    acc_y[k] += s_d[(pty * VP + ptx) * 10 + 5 + a];
                }
            } else {
#pragma unroll
                for (int a = 0; a < 5; a += 2) {
                    const int ptx = (qa - a) / 2 + 2;
                    acc_x[k] += s_d[(pty * VP + ptx) * 10 + a];
                    acc_y[k] += s_d[(pty * VP + ptx) * 10 + 5 + a];
                }
            }
        }
        __syncthreads();
    }
    const T dp = row_dot(M + 50 * kSlots, rv);
#pragma unroll
    for (int k = 0; k < VOWN_PER_THREAD; ++k) {
        const int q = tid + k * VNT;
        if (q >= VOWN * VOWN) continue;
        const int gi = 2 * E0x + q % VOWN, gj = 2 * E0y + q / VOWN;
        if (gi >= g.s2 - 1 || gj >= g.s2 - 1 || gi == 0 || gj == 0) continue;
        const int64_t qq = int64_t(gj) * g.s2 + gi;
        x[qq] += acc_x[k];
        x[g.nq2 + qq] += acc_y[k];
    }
    if (valid && tx >= 1 && tx <= VT && ty >= 1 && ty <= VT)
        x[2 * g.nq2 + int64_t(J) * g.s1 + I] += dp;
}

// ---------------------------------------------------------------------------
// Transfers
// ---------------------------------------------------------------------------

// 1D restriction weights of coarse Q2 node ic from fine offsets.
__device__ __forceinline__ int q2_restrict_taps(int ic, int (&off)[5], double (&w)[5]) {
    if ((ic & 1) == 0) {
        off[0] = -3; w[0] = -0.125;
        off[1] = -1; w[1] = 0.375;
        off[2] = 0;  w[2] = 1.0;
        off[3] = 1;  w[3] = 0.375;
        off[4] = 3;  w[4] = -0.125;
        return 5;
    }
    off[0] = -1; w[0] = 0.75;
    off[1] = 0;  w[1] = 1.0;
    off[2] = 1;  w[2] = 0.75;
    return 3;
}

template <typename T>
__global__ __launch_bounds__(256) void restrict_kernel(Geom gf, Geom gc, const T* __restrict__ rf,
                                                       T* __restrict__ bc) {
    const int ic = blockIdx.x * 16 + (threadIdx.x & 15);
    const int jc = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (ic < gc.s2 && jc < gc.s2) {
        const int64_t qc = int64_t(jc) * gc.s2 + ic;
        T sx = 0, sy = 0;
        if (!q2_boundary(ic, jc, gc.s2)) {
            int ox[5], oy[5];
            double wx[5], wy[5];
            const int nx = q2_restrict_taps(ic, ox, wx);
            const int ny = q2_restrict_taps(jc, oy, wy);
            for (int b = 0; b < ny; ++b) {
                const int jf = 2 * jc + oy[b];
                T tx = 0, ty = 0;
                for (int a = 0; a < nx; ++a) {
                    const int i_f = 2 * ic + ox[a];
                    if (q2_boundary(i_f, jf, gf.s2)) continue;
                    const int64_t qf = int64_t(jf) * gf.s2 + i_f;
                    tx += T(wx[a]) * rf[qf];
                    ty += T(wx[a]) * rf[gf.nq2 + qf];
                }
                sx += T(wy[b]) * tx;
                sy += T(wy[b]) * ty;
            }
        }
        bc[qc] = sx;
        bc[gc.nq2 + qc] = sy;
    }
    if (ic < gc.s1 && jc < gc.s1) {
        T s = 0;
        for (int oyy = -1; oyy <= 1; ++oyy) {
            const int jf = 2 * jc + oyy;
            if (jf < 0 || jf >= gf.s1) continue;
            const T wy = oyy == 0 ? T(1) : T(0.5);
            T t = 0;
            for (int oxx = -1; oxx <= 1; ++oxx) {
                const int i_f = 2 * ic + oxx;
                if (i_f < 0 || i_f >= gf.s1) continue;
                const T wx = oxx == 0 ? T(1) : T(0.5);
                t += wx * rf[2 * gf.nq2 + int64_t(jf) * gf.s1 + i_f];
            }
            s += wy * t;
        }
        bc[2 * gc.nq2 + int64_t(jc) * gc.s1 + ic] = s;
    }
}

// 1D interpolation taps of fine Q2 node i from coarse Q2 nodes.
__device__ __forceinline__ int q2_prolong_taps(int i, int (&c)[3], double (&w)[3]) {
    if ((i & 1) == 0) {
        c[0] = i / 2; w[0] = 1.0;
        return 1;
    }
    const int e = i / 4;  // coarse element
    c[0] = 2 * e; c[1] = 2 * e + 1; c[2] = 2 * e + 2;
    if ((i & 3) == 1) {
        w[0] = 0.375; w[1] = 0.75; w[2] = -0.125;
    } else {
        w[0] = -0.125; w[1] = 0.75; w[2] = 0.375;
    }
    return 3;
}

template <typename T>
__global__ __launch_bounds__(256) void prolong_kernel(Geom gf, Geom gc, const T* __restrict__ ec,
                                                      T* __restrict__ xf) {
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i < gf.s2 && j < gf.s2 && !q2_boundary(i, j, gf.s2)) {
        int cx[3], cy[3];
        double wx[3], wy[3];
        const int nx = q2_prolong_taps(i, cx, wx);
        const int ny = q2_prolong_taps(j, cy, wy);
        T sx = 0, sy = 0;
        for (int b = 0; b < ny; ++b) {
            T tx = 0, ty = 0;
            for (int a = 0; a < nx; ++a) {
                if (q2_boundary(cx[a], cy[b], gc.s2)) continue;
                const int64_t qc = int64_t(cy[b]) * gc.s2 + cx[a];
                tx += T(wx[a]) * ec[qc];
                ty += T(wx[a]) * ec[gc.nq2 + qc];
            }
            sx += T(wy[b]) * tx;
            sy += T(wy[b]) * ty;
        }
        const int64_t q = int64_t(j) * gf.s2 + i;
        xf[q] += sx;
        xf[gf.nq2 + q] += sy;
    }
    if (i < gf.s1 && j < gf.s1) {
        const int i0 = i / 2, i1 = (i + 1) / 2, j0 = j / 2, j1 = (j + 1) / 2;
        const T* pc = ec + 2 * gc.nq2;
        T v;
        if ((i & 1) == 0 && (j & 1) == 0) {
            v = pc[int64_t(j0) * gc.s1 + i0];
        } else if ((j & 1) == 0) {
            v = T(0.5) * (pc[int64_t(j0) * gc.s1 + i0] + pc[int64_t(j0) * gc.s1 + i1]);
        } else if ((i & 1) == 0) {
            v = T(0.5) * (pc[int64_t(j0) * gc.s1 + i0] + pc[int64_t(j1) * gc.s1 + i0]);
        } else {
            v = T(0.25) * ((pc[int64_t(j0) * gc.s1 + i0] + pc[int64_t(j0) * gc.s1 + i1]) +
                           (pc[int64_t(j1) * gc.s1 + i0] + pc[int64_t(j1) * gc.s1 + i1]));
        }
        xf[2 * gf.nq2 + int64_t(j) * gf.s1 + i] += v;
    }
}

// ---------------------------------------------------------------------------
// Coarse solve: e = C r, one wavefront per row, FP64 accumulation.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
__global__ __launch_bounds__(256) void coarse_gemv_kernel(int64_t n, const double* __restrict__ C,
                                                          const T* __restrict__ r,
                                                          T* __restrict__ e) {
    const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    double s = 0.0;
    for (int64_t c = lane; c < n; c += 64) s += C[row * n + c] * double(r[c]);
    s = wave_sum(s);
    if (lane == 0) e[row] = T(s);
}

// ---------------------------------------------------------------------------
// Elementwise
// ---------------------------------------------------------------------------

template <typename T>
__global__ void fill_zero_kernel(T* __restrict__ x, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        x[i] = T(0);
}

template <typename Ti, typename To>
__global__ void cast_kernel(const Ti* __restrict__ in, To* __restrict__ out, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = To(in[i]);
}

__global__ void scale_kernel(const double* __restrict__ in, double alpha, double* __restrict__ out,
                             int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = alpha * in[i];
}

// ---------------------------------------------------------------------------
// Krylov: multi-dot, reduction, update, multi-axpy
// ---------------------------------------------------------------------------

template <int KMAX>
__global__ __launch_bounds__(256) void mdot_partial_kernel(const double* __restrict__ V,
                                                           int64_t ldv, int k,
                                                           const double* __restrict__ w,
                                                           int64_t n,
                                                           double* __restrict__ part) {
    double acc[KMAX];
#pragma unroll
    for (int v = 0; v < KMAX; ++v) acc[v] = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        const double wi = w[i];
#pragma unroll
        for (int v = 0; v < KMAX; ++v)
            if (v < k) acc[v] += V[v * ldv + i] * wi;
    }
    __shared__ double red[KMAX][4];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < KMAX; ++v) {
        const double s = wave_sum(acc[v]);
        if (lane == 0) red[v][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < k)
        part[int64_t(threadIdx.x) * gridDim.x + blockIdx.x] =
            (red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]);
}

__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ part,
                                                              int nblk,
                                                              double* __restrict__ out) {
    const int v = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) s += part[int64_t(v) * nblk + i];
    __shared__ double red[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[v] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <int KMAX>
__global__ __launch_bounds__(256) void update_kernel(const double* __restrict__ V, int64_t ldv,
                                                     int k, const double* __restrict__ h,
                                                     double* __restrict__ w, int64_t n,
                                                     double* __restrict__ part) {
    double hv[KMAX];
#pragma unroll
    for (int v = 0; v < KMAX; ++v) hv[v] = v < k ? h[v] : 0.0;
    double nrm = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        double s = w[i];
#pragma unroll
        for (int v = 0; v < KMAX; ++v)
            if (v < k) s -= hv[v] * V[v * ldv + i];
        w[i] = s;
        nrm += s * s;
    }
    if (part != nullptr) {
        __shared__ double red[4];
        nrm = wave_sum(nrm);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
        __syncthreads();
        if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

template <int KMAX>
__global__ __launch_bounds__(256) void axpy_multi_kernel(const double* __restrict__ Z, int64_t ldz,
                                                         int k, const double* __restrict__ y,
                                                         double* __restrict__ x, int64_t n) {
    double yv[KMAX];
#pragma unroll
    for (int v = 0; v < KMAX; ++v) yv[v] = v < k ? y[v] : 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        double s = x[i];
#pragma unroll
        for (int v = 0; v < KMAX; ++v)
            if (v < k) s += yv[v] * Z[v * ldz + i];
        x[i] = s;
    }
}

int elementwise_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return int(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <typename Tx, typename T>
void launch_residual(const Geom& g, const T* b, const Tx* x, T* r, int mode, hipStream_t s) {
    const dim3 grid((g.N + 1 + 15) / 16, (g.N + 1 + 15) / 16);
    if (mode == 0)
        residual_kernel<0, Tx, T><<<grid, 256, 0, s>>>(g, b, x, r);
    else
        residual_kernel<1, Tx, T><<<grid, 256, 0, s>>>(g, b, x, r);
}
template void launch_residual<double, double>(const Geom&, const double*, const double*, double*,
                                              int, hipStream_t);
template void launch_residual<float, float>(const Geom&, const float*, const float*, float*, int,
                                            hipStream_t);

void launch_rhs(const Geom& g, const double* f, const double* gd, double* b, hipStream_t s) {
    const dim3 grid((g.N + 1 + 15) / 16, (g.N + 1 + 15) / 16);
    rhs_kernel<<<grid, 256, 0, s>>>(g, f, gd, b);
}

template <typename T>
void launch_vanka_update(const Geom& g, const T* r, T* x, const T* Wall, hipStream_t s) {
    const int tiles = (g.N + 1 + VT - 1) / VT;
    const TileRange ir = interior_tiles(g.N);
    const int ni = ir.hi - ir.lo;
    if (ni > 0) vanka_update_kernel<T, true><<<dim3(ni, ni), VNT, 0, s>>>(g, r, x, Wall);
    vanka_update_kernel<T, false><<<dim3(tiles, tiles), VNT, 0, s>>>(g, r, x, Wall);
}
template void launch_vanka_update<double>(const Geom&, const double*, double*, const double*,
                                          hipStream_t);
template void launch_vanka_update<float>(const Geom&, const float*, float*, const float*,
                                         hipStream_t);

template <typename T>
void launch_restrict(const Geom& gf, const Geom& gc, const T* rf, T* bc, hipStream_t s) {
    const dim3 grid((gc.s2 + 15) / 16, (gc.s2 + 15) / 16);
    restrict_kernel<T><<<grid, 256, 0, s>>>(gf, gc, rf, bc);
}
template void launch_restrict<double>(const Geom&, const Geom&, const double*, double*, hipStream_t);
template void launch_restrict<float>(const Geom&, const Geom&, const float*, float*, hipStream_t);

template <typename T>
void launch_prolong_add(const Geom& gf, const Geom& gc, const T* ec, T* xf, hipStream_t s) {
    const dim3 grid((gf.s2 + 15) / 16, (gf.s2 + 15) / 16);
    prolong_kernel<T><<<grid, 256, 0, s>>>(gf, gc, ec, xf);
}
template void launch_prolong_add<double>(const Geom&, const Geom&, const double*, double*,
                                         hipStream_t);
template void launch_prolong_add<float>(const Geom&, const Geom&, const float*, float*,
                                        hipStream_t);

template <typename T>
void launch_coarse_gemv(int64_t n, const double* C, const T* r, T* e, hipStream_t s) {
    coarse_gemv_kernel<T><<<int((n + 3) / 4), 256, 0, s>>>(n, C, r, e);
}
template void launch_coarse_gemv<double>(int64_t, const double*, const double*, double*,
                                         hipStream_t);
template void launch_coarse_gemv<float>(int64_t, const double*, const float*, float*, hipStream_t);

template <typename T>
void launch_fill_zero(T* x, int64_t n, hipStream_t s) {
    fill_zero_kernel<T><<<elementwise_blocks(n), 256, 0, s>>>(x, n);
}
template void launch_fill_zero<double>(double*, int64_t, hipStream_t);
template void launch_fill_zero<float>(float*, int64_t, hipStream_t);

template <typename Ti, typename To>
void launch_cast(const Ti* in, To* out, int64_t n, hipStream_t s) {
    cast_kernel<Ti, To><<<elementwise_blocks(n), 256, 0, s>>>(in, out, n);
}
template void launch_cast<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_cast<float, double>(const float*, double*, int64_t, hipStream_t);

void launch_scale(const double* in, double alpha, double* out, int64_t n, hipStream_t s) {
    scale_kernel<<<elementwise_blocks(n), 256, 0, s>>>(in, alpha, out, n);
}

#define VKMG_KDISPATCH(k, KERNEL, ...)                              \
    do {                                                            \
        if ((k) <= 4) KERNEL<4><<<kDotBlocks, 256, 0, s>>>(__VA_ARGS__);        \
        else if ((k) <= 8) KERNEL<8><<<kDotBlocks, 256, 0, s>>>(__VA_ARGS__);   \
        else if ((k) <= 16) KERNEL<16><<<kDotBlocks, 256, 0, s>>>(__VA_ARGS__); \
        else KERNEL<32><<<kDotBlocks, 256, 0, s>>>(__VA_ARGS__);                \
    } while (0)

// The Krylov kernels keep up to 32 coefficients in registers; longer
// bases are processed in chunks of 32 vectors.
constexpr int kChunk = 32;

void launch_mdot_partial(const double* V, int64_t ldv, int k, const double* w, int64_t n,
                         double* part, hipStream_t s) {
    for (int c0 = 0; c0 < k; c0 += kChunk) {
        const int kc = k - c0 < kChunk ? k - c0 : kChunk;
        VKMG_KDISPATCH(kc, mdot_partial_kernel, V + c0 * ldv, ldv, kc, w, n,
                       part + int64_t(c0) * kDotBlocks);
    }
}

void launch_reduce_partials(const double* part, int k, double* out, hipStream_t s) {
    reduce_partials_kernel<<<k, 256, 0, s>>>(part, kDotBlocks, out);
}

void launch_update(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t n,
                   double* part, hipStream_t s) {
    for (int c0 = 0; c0 < k; c0 += kChunk) {
        const int kc = k - c0 < kChunk ? k - c0 : kChunk;
        double* pp = (c0 + kc >= k) ? part : nullptr;  // norm after the last chunk
        VKMG_KDISPATCH(kc, update_kernel, V + c0 * ldv, ldv, kc, h + c0, w, n, pp);
    }
}

void launch_axpy_multi(const double* Z, int64_t ldz, int k, const double* y, double* x, int64_t n,
                       hipStream_t s) {
    for (int c0 = 0; c0 < k; c0 += kChunk) {
        const int kc = k - c0 < kChunk ? k - c0 : kChunk;
        VKMG_KDISPATCH(kc, axpy_multi_kernel, Z + c0 * ldz, ldz, kc, y + c0, x, n);
    }
}

}  // namespace vkmg
