// HIP kernels of the vkmg library for gfx950 (CDNA4, wave64).
//
// Layout of every level vector: [u_x | u_y | p], Q2 blocks of (2N+1)^2 and a
// Q1 block of (N+1)^2 values, row-major (index j*side + i).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "kernels.h"
#include "stencil.h"
#include "interior_blocks.h"
#include "symmetry.h"
#include "mfma_patch.h"
#include "d4_apply.h"

namespace vkmg {

namespace {

__device__ __forceinline__ bool q2_boundary(int qi, int qj, int s2) {
    return qi == 0 || qj == 0 || qi == s2 - 1 || qj == s2 - 1;
}

// ---------------------------------------------------------------------------
// Rows of A for one cell from LDS-staged values.  A cell (ex, ey) holds the
// Q2 nodes (2ex+a, 2ey+b), a, b in {0,1}, and the Q1 node (ex, ey).  The
// staged velocity arrays (row stride SQ2) hold x with Dirichlet columns and
// outside nodes already zeroed; c2 is the staged index of node (2ex, 2ey);
// the staged pressure array (row stride SQ1) has c1 at Q1 node (ex, ey).
// cell_row_pair<.., BB> returns (A x) at the two Q2 nodes of row parity BB
// (both components; meaningful for free nodes) and, for BB = 0, (B u) at
// the Q1 node.
// ---------------------------------------------------------------------------

template <int SQ2, int SQ1, int BB, typename T>
__device__ __forceinline__ void cell_row_pair(const T* __restrict__ su0, const T* __restrict__ su1,
                                              const T* __restrict__ sp, int c2, int c1, T cl, T cb,
                                              T (&ax)[2], T (&ay)[2], T& ap) {
#pragma unroll
    for (int aa = 0; aa < 2; ++aa) {
        T lx = 0, ly = 0, bx = 0, by = 0;
        const int cn = c2 + BB * SQ2 + aa;
#pragma unroll
        for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
            for (int dx = -2; dx <= 2; ++dx) {
                const int c = st_L(BB, aa, dy, dx);
                if (c != 0) {
                    lx += T(c) * su0[cn + dy * SQ2 + dx];
                    ly += T(c) * su1[cn + dy * SQ2 + dx];
                }
            }
        // B^T p: Q1 nodes I with offsets o = i - 2I of the parity of i
#pragma unroll
        for (int oy = -2; oy <= 2; ++oy) {
            if (((oy - BB) & 1) != 0) continue;
#pragma unroll
            for (int oxx = -2; oxx <= 2; ++oxx) {
                if (((oxx - aa) & 1) != 0) continue;
                const int cx = st_Mq(oy) * st_G(oxx);
                const int cy = st_G(oy) * st_Mq(oxx);
                if (cx == 0 && cy == 0) continue;
                const T pv = sp[c1 + ((BB - oy) / 2) * SQ1 + (aa - oxx) / 2];
                bx += T(cx) * pv;
                by += T(cy) * pv;
            }
        }
        ax[aa] = cl * lx + cb * bx;
        ay[aa] = cl * ly + cb * by;
    }
    ap = 0;
    if (BB == 0) {
        T sp_ = 0;
#pragma unroll
        for (int oy = -2; oy <= 2; ++oy)
#pragma unroll
            for (int oxx = -2; oxx <= 2; ++oxx) {
                const int cx = st_Mq(oy) * st_G(oxx);
                const int cy = st_G(oy) * st_Mq(oxx);
                if (cx == 0 && cy == 0) continue;
                const int cc = c2 + oy * SQ2 + oxx;
                sp_ += T(cx) * su0[cc] + T(cy) * su1[cc];
            }
        ap = cb * sp_;
    }
}

// 1D interpolation taps of fine Q2 node i from coarse Q2 nodes, padded to
// three (a fine node on a coarse node has one tap of weight 1).
__device__ __forceinline__ void q2_prolong_taps(int i, int (&c)[3], double (&w)[3]) {
    if ((i & 1) == 0) {
        c[0] = i / 2; w[0] = 1.0;
        c[1] = i / 2; w[1] = 0.0;
        c[2] = i / 2; w[2] = 0.0;
        return;
    }
    const int e = i / 4;  // coarse element
    c[0] = 2 * e; c[1] = 2 * e + 1; c[2] = 2 * e + 2;
    if ((i & 3) == 1) {
        w[0] = 0.375; w[1] = 0.75; w[2] = -0.125;
    } else {
        w[0] = -0.125; w[1] = 0.75; w[2] = 0.375;
    }
}

// ---------------------------------------------------------------------------
// Residual r = b - A x (MODE 0) / apply r = A x (MODE 1)
// A workgroup computes the rows of a tile of RT x RT cells, one thread per
// cell; x on the Q2 nodes within two of the tile and the Q1 nodes within
// one is staged in LDS with the Dirichlet columns zeroed, so that every row
// is a fixed stencil.
// ---------------------------------------------------------------------------

constexpr int RT = 16;              // cells per tile side
constexpr int RQ2 = 2 * RT + 4;     // staged Q2 nodes per side
constexpr int RQ1 = RT + 2;         // staged Q1 nodes per side
constexpr int RNT = 2 * RT * RT;    // threads: one per cell and Q2 row parity

// 1D Q2 stiffness (x 1/(3h)) and mass (x h/30) of one element, local nodes
// 0, 1 (midpoint), 2: the element Laplacian per unit viscosity between
// local nodes (a,b) and (c,d) is (M[b][d] K[a][c] + K[b][d] M[a][c]) / 90.
__device__ constexpr int kEK[3][3] = {{7, -8, 1}, {-8, 16, -8}, {1, -8, 7}};
__device__ constexpr int kEM[3][3] = {{4, 2, -1}, {2, 16, 2}, {-1, 2, 4}};

// Stage x + P ec for a residual tile (Q2 nodes [2E0 - 2, 2E0 + RQ2 - 2) and
// Q1 nodes [E0 - 1, E0 + RQ1 - 1) per direction; Dirichlet and outside
// nodes zero, as the residual staging).  Q2: one item per staged column
// and coarse element row, interpolating along x and then y with the
// expressions of prolong_kernel; Q1: bilinear per node, likewise.  A
// thread takes at most one item and one Q1 node and issues all their loads
// before the first is used.
constexpr int kProRows = RQ2 / 4 + 1;  // coarse element rows meeting the staged rows
static_assert(RQ2 * kProRows <= RNT && RQ1 * RQ1 <= RNT, "one staging item per thread");

template <typename T>
__device__ __forceinline__ void stage_prolonged(const Geom& g, const Geom& gc, const T* x,
                                                const T* ec, int E0x, int E0y, T* su0, T* su1,
                                                T* sp) {
    const int ox = 2 * E0x - 2, oy = 2 * E0y - 2;
    const int jg0 = (oy + 4) / 4 - 1;  // floor(oy / 4), oy >= -2
    const int item = threadIdx.x;
    const bool q2item = item < RQ2 * kProRows;
    const int ci = item % RQ2, jg = jg0 + item / RQ2;
    const int i = ox + ci;
    const bool col = q2item && i >= 0 && i < g.s2 && jg >= 0 && jg < gc.N;
    int cx[3];
    double wx[3];
    q2_prolong_taps(col ? i : 0, cx, wx);
    T f0[4], f1[4], vx[3][3], vy[3][3];
    bool fr[4], ok[3][3];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int fj = 4 * jg + p;
        fr[p] = col && i > 0 && i < g.s2 - 1 && fj > 0 && fj < g.s2 - 1;
        const int64_t q = fr[p] ? int64_t(fj) * g.s2 + i : 0;
        f0[p] = x[q];
        f1[p] = x[g.nq2 + q];
    }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ok[b][a] = col && !q2_boundary(cx[a], 2 * jg + b, gc.s2);
            const int64_t qc = ok[b][a] ? int64_t(2 * jg + b) * gc.s2 + cx[a] : 0;
            vx[b][a] = ec[qc];
            vy[b][a] = ec[gc.nq2 + qc];
        }
    // Q1 node t = threadIdx.x
    const int t = threadIdx.x;
    const int I = E0x - 1 + t % RQ1, J = E0y - 1 + t / RQ1;
    const bool pin = t < RQ1 * RQ1 && I >= 0 && J >= 0 && I <= g.N && J <= g.N;
    const int Ic = pin ? I : 0, Jc = pin ? J : 0;
    const int i0 = Ic / 2, i1 = (Ic + 1) / 2, j0 = Jc / 2, j1 = (Jc + 1) / 2;
    const T* pc = ec + 2 * gc.nq2;
    const T fp = x[2 * g.nq2 + int64_t(Jc) * g.s1 + Ic];
    const T p00 = pc[int64_t(j0) * gc.s1 + i0], p01 = pc[int64_t(j0) * gc.s1 + i1];
    const T p10 = pc[int64_t(j1) * gc.s1 + i0], p11 = pc[int64_t(j1) * gc.s1 + i1];

    T tx[3], ty[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        tx[b] = 0;
        ty[b] = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T wa = ok[b][a] ? T(wx[a]) : T(0);
            tx[b] += wa * vx[b][a];
            ty[b] += wa * vy[b][a];
        }
    }
    const T sx[4] = {tx[0], T(0.375) * tx[0] + T(0.75) * tx[1] + T(-0.125) * tx[2], tx[1],
                     T(-0.125) * tx[0] + T(0.75) * tx[1] + T(0.375) * tx[2]};
    const T sy[4] = {ty[0], T(0.375) * ty[0] + T(0.75) * ty[1] + T(-0.125) * ty[2], ty[1],
                     T(-0.125) * ty[0] + T(0.75) * ty[1] + T(0.375) * ty[2]};
    if (q2item) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int lr = 4 * jg + p - oy;
            if (lr < 0 || lr >= RQ2) continue;
            su0[lr * RQ2 + ci] = fr[p] ? f0[p] + sx[p] : T(0);
            su1[lr * RQ2 + ci] = fr[p] ? f1[p] + sy[p] : T(0);
        }
    }
    if (t < RQ1 * RQ1) {
        const T r0 = (Ic & 1) ? T(0.5) * (p00 + p01) : p00;
        const T r1 = (Ic & 1) ? T(0.5) * (p10 + p11) : p10;
        sp[t] = pin ? fp + ((Jc & 1) ? T(0.5) * (r0 + r1) : r0) : T(0);
    }
}

// VAR: per-element viscosity nue (N^2 values, index ey*N + ex); the L rows
// are then summed element by element (each Q2 node lies in 1, 2 or 4
// elements) instead of by the constant-coefficient stencil.
// PRO (MODE 0, Tx = T): the coarse-grid correction is added first: the tile
// stages x + P ec (ec on the coarse level gc, the arithmetic of
// prolong_kernel, so the sums are the same), writes it to x2 for the nodes
// whose rows it computes, and forms r = b - A (x + P ec).
// COPY: x converted to T is also written to x2 for those nodes (an FP32 x
// widened to FP64 next to its FP64 operator apply).
template <int MODE, typename Tx, typename T, bool VAR = false, bool PRO = false, bool COPY = false>
__global__ __launch_bounds__(RNT) __attribute__((amdgpu_waves_per_eu(4))) void residual_kernel(Geom g, const T* __restrict__ b,
                                                       const Tx* __restrict__ x,
                                                       T* __restrict__ r,
                                                       const T* __restrict__ nue = nullptr,
                                                       Geom gc = Geom{},
                                                       const T* __restrict__ ec = nullptr,
                                                       T* __restrict__ x2 = nullptr) {
    __shared__ T s_u[2][RQ2 * RQ2];
    __shared__ T s_p[RQ1 * RQ1];
    __shared__ T s_nu[VAR ? RQ1 * RQ1 : 1];
    const int tiles = (g.N + 1 + RT - 1) / RT;
    const int ntile = tiles * tiles;
    const int per_xcd = (ntile + 7) / 8;
    const int tlin = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tlin >= ntile) return;
    {  // right-hand side blockIdx.y of a batch (vectors g.n apart)
        const int64_t bo = int64_t(blockIdx.y) * g.n;
        if (MODE == 0) b += bo;
        x += bo;
        r += bo;
        if (PRO || COPY) x2 += bo;
        if (PRO) ec += int64_t(blockIdx.y) * gc.n;
    }
    const int E0x = (tlin % tiles) * RT, E0y = (tlin / tiles) * RT;
    const int ox = 2 * E0x - 2, oy = 2 * E0y - 2;
    if constexpr (PRO) {
        stage_prolonged(g, gc, x, ec, E0x, E0y, s_u[0], s_u[1], s_p);
    } else {
    // every load of the tile is issued before the first is used: addresses
    // of nodes outside the staged set are clamped to node 0 and the values
    // replaced by zero afterwards
    constexpr int kIt2 = (RQ2 * RQ2 + RNT - 1) / RNT, kIt1 = (RQ1 * RQ1 + RNT - 1) / RNT;
    Tx v0[kIt2], v1[kIt2], vp[kIt1];
    bool f2[kIt2], f1[kIt1];
#pragma unroll
    for (int it = 0; it < kIt2; ++it) {
        const int t = threadIdx.x + it * RNT;
        const int qi = ox + t % RQ2, qj = oy + t / RQ2;
        f2[it] = t < RQ2 * RQ2 && qi > 0 && qj > 0 && qi < g.s2 - 1 && qj < g.s2 - 1;
        const int64_t q = f2[it] ? int64_t(qj) * g.s2 + qi : 0;
        v0[it] = x[q];
        v1[it] = x[g.nq2 + q];
    }
#pragma unroll
    for (int it = 0; it < kIt1; ++it) {
        const int t = threadIdx.x + it * RNT;
        const int I = E0x - 1 + t % RQ1, J = E0y - 1 + t / RQ1;
        f1[it] = t < RQ1 * RQ1 && I >= 0 && J >= 0 && I <= g.N && J <= g.N;
        vp[it] = x[2 * g.nq2 + (f1[it] ? int64_t(J) * g.s1 + I : 0)];
    }
#pragma unroll
    for (int it = 0; it < kIt2; ++it) {
        const int t = threadIdx.x + it * RNT;
        if (t < RQ2 * RQ2) {
            s_u[0][t] = f2[it] ? T(v0[it]) : T(0);
            s_u[1][t] = f2[it] ? T(v1[it]) : T(0);
        }
    }
#pragma unroll
    for (int it = 0; it < kIt1; ++it) {
        const int t = threadIdx.x + it * RNT;
        if (t < RQ1 * RQ1) s_p[t] = f1[it] ? T(vp[it]) : T(0);
    }
    }
    if (VAR) {  // viscosities of the elements [E0-1, E0+RT] per direction
        for (int t = threadIdx.x; t < RQ1 * RQ1; t += RNT) {
            const int ex = E0x - 1 + t % RQ1, ey = E0y - 1 + t / RQ1;
            const bool in = ex >= 0 && ey >= 0 && ex < g.N && ey < g.N;
            s_nu[t] = in ? nue[int64_t(ey) * g.N + ex] : T(0);
        }
    }
    __syncthreads();
    // this thread: the two Q2 nodes of row parity bb of cell (tx, ty) (and
    // for bb = 0 the cell's Q1 node); waves 0-3 take bb = 0, waves 4-7 bb = 1
    const int bb = threadIdx.x / (RT * RT);
    const int cidx = threadIdx.x % (RT * RT);
    const int tx = cidx % RT, ty = cidx / RT;
    const int ex = E0x + tx, ey = E0y + ty;
    const bool cell = ex <= g.N && ey <= g.N;
    int64_t qn[2];
    T bx[2], by[2];
#pragma unroll
    for (int aa = 0; aa < 2; ++aa) {
        const int i = 2 * ex + aa, j = 2 * ey + bb;
        qn[aa] = (cell && i < g.s2 && j < g.s2) ? int64_t(j) * g.s2 + i : -1;
        const int64_t q = qn[aa] >= 0 ? qn[aa] : 0;
        if (MODE == 0) {
            bx[aa] = b[q];
            by[aa] = b[g.nq2 + q];
        }
    }
    const int64_t qp = 2 * g.nq2 + (cell ? int64_t(ey) * g.s1 + ex : 0);
    const T bp = (MODE == 0 && bb == 0) ? b[qp] : T(0);
    if (!cell) return;
    T ax[2], ay[2], ap;
    const int c2 = (2 * ty + 2) * RQ2 + 2 * tx + 2, c1 = (ty + 1) * RQ1 + tx + 1;
    const T cl = T(g.nu / 90.0), cb = T(-g.h / 36.0);
    if (bb == 0)
        cell_row_pair<RQ2, RQ1, 0>(s_u[0], s_u[1], s_p, c2, c1, VAR ? T(0) : cl, cb, ax, ay, ap);
    else
        cell_row_pair<RQ2, RQ1, 1>(s_u[0], s_u[1], s_p, c2, c1, VAR ? T(0) : cl, cb, ax, ay, ap);
    if (VAR) {
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) {
            T lx = 0, ly = 0;
            // elements containing node (2ex+aa, 2ey+bb): ex-1 and ex for a
            // vertex column (aa = 0), ex for a midpoint column; same in y
#pragma unroll
            for (int ey_ = -1; ey_ <= 0; ++ey_) {
                if (bb == 1 && ey_ == -1) continue;
#pragma unroll
                for (int ex_ = -1; ex_ <= 0; ++ex_) {
                    if (aa == 1 && ex_ == -1) continue;
                    const int la = aa - 2 * ex_, lb = bb - 2 * ey_;  // local node
                    const T nv = s_nu[(ty + 1 + ey_) * RQ1 + tx + 1 + ex_];
                    T ex0 = 0, ey0 = 0;
#pragma unroll
                    for (int d = 0; d < 3; ++d)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const int co = kEM[lb][d] * kEK[la][c] + kEK[lb][d] * kEM[la][c];
                            if (co == 0) continue;
                            const int cc = c2 + (2 * ey_ + d) * RQ2 + 2 * ex_ + c;
                            ex0 += T(co) * s_u[0][cc];
                            ey0 += T(co) * s_u[1][cc];
                        }
                    lx += nv * ex0;
                    ly += nv * ey0;
                }
            }
            ax[aa] += T(1.0 / 90.0) * lx;
            ay[aa] += T(1.0 / 90.0) * ly;
        }
    }
#pragma unroll
    for (int aa = 0; aa < 2; ++aa) {
        const int64_t q = qn[aa];
        if (q < 0) continue;
        const int i = 2 * ex + aa, j = 2 * ey + bb;
        T vx = ax[aa], vy = ay[aa];
        const bool dir = i == 0 || j == 0 || i == g.s2 - 1 || j == g.s2 - 1;
        if (dir) {
            vx = T(x[q]);  // Dirichlet row: identity (edge tiles only)
            vy = T(x[g.nq2 + q]);
        }
        if (PRO || COPY) {  // x + P ec (PRO) or x (COPY); Dirichlet: x
            x2[q] = dir ? T(x[q]) : s_u[0][c2 + bb * RQ2 + aa];
            x2[g.nq2 + q] = dir ? T(x[g.nq2 + q]) : s_u[1][c2 + bb * RQ2 + aa];
        }
        if (MODE == 0) {
            r[q] = bx[aa] - vx;
            r[g.nq2 + q] = by[aa] - vy;
        } else {
            r[q] = vx;
            r[g.nq2 + q] = vy;
        }
    }
    if (bb == 0) r[qp] = (MODE == 0) ? bp - ap : ap;
    if ((PRO || COPY) && bb == 0) x2[qp] = s_p[c1];
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
    {  // right-hand side blockIdx.z of a batch
        const int64_t z = blockIdx.z;
        f += z * 2 * g.nq2;
        if (gd) gd += z * 2 * g.nq2;
        b += z * g.n;
    }
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
// Braess-Sarazin relaxation (inexact form): with D = diag(L) and
// S = -(1/t) B D^{-1} B^T,
//   rhs = r_p - (1/t) B D^{-1} r_u,  dp = Jacobi sweeps on S dp = rhs,
//   x_u += w (1/t) D^{-1} (r_u - B^T dp),  x_p += w dp.
// Tiles of BT x BT cells, one thread per cell (its Q1 node and its Q2 nodes
// (2ex+a, 2ey+b)); D^{-1} and diag(S) are formed in the kernels from the
// stencil constants (free velocity DoFs: D = (nu/90) L-stencil centre;
// Dirichlet DoFs: identity rows, no B coupling).
// ---------------------------------------------------------------------------

constexpr int BT = 16;            // cells per tile side
constexpr int BQ2 = 2 * BT + 4;   // staged Q2 nodes per side (offset -2)
constexpr int BQ1 = BT + 2;       // staged Q1 nodes per side (offset -1)
constexpr int BNT = BT * BT;

template <typename T>
__device__ __forceinline__ T bs_dinv(const Geom& g, int px, int py) {
    return T(1.0 / (g.nu / 90.0 * double(st_L(py, px, 0, 0))));
}

// diag(S) at Q1 node (I, J): -(1/t) sum over the free Q2 nodes j of the
// patch of B_Ij^2 / D_j (both components).
template <typename T>
__device__ __forceinline__ T bs_schur_diag(const Geom& g, int I, int J, T inv_t) {
    const double cb = -g.h / 36.0, cl = g.nu / 90.0;
    double s = 0.0;
#pragma unroll
    for (int oy = -2; oy <= 2; ++oy)
#pragma unroll
        for (int ox = -2; ox <= 2; ++ox) {
            const int cx = st_Mq(oy) * st_G(ox), cy = st_G(oy) * st_Mq(ox);
            if (cx == 0 && cy == 0) continue;
            const int qi = 2 * I + ox, qj = 2 * J + oy;
            const bool free = qi > 0 && qj > 0 && qi < g.s2 - 1 && qj < g.s2 - 1;
            const double d = cl * double(st_L(oy & 1, ox & 1, 0, 0));
            s += free ? double(cx * cx + cy * cy) / d : 0.0;
        }
    return T(-double(inv_t) * cb * cb * s);
}

// MODE 0: prhs = vin_p - (1/t) B D^{-1} vin_u (vin = the residual r),
// dp = wj prhs / diag(S).
// MODE 1: dp += wj (prhs + (1/t) B D^{-1} vin_u) / diag(S) (vin_u = B^T dp of
// the previous Jacobi iterate, so that the bracket is prhs - S dp).
// Batched over blockIdx.y: vin advances by g.n (MODE 0) or 2 nq2 (MODE 1),
// prhs and dp by g.nq1.
template <typename T, int MODE>
__global__ __launch_bounds__(BNT) void bs_div_kernel(Geom g, const T* vin, T* prhs, T* dp,
                                                     T inv_t, T wj) {
    __shared__ T s_u[2][BQ2 * BQ2];
    const int tiles = (g.N + 1 + BT - 1) / BT;
    const int ntile = tiles * tiles;
    const int per_xcd = (ntile + 7) / 8;
    const int tlin = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tlin >= ntile) return;
    vin += int64_t(blockIdx.y) * (MODE == 0 ? g.n : 2 * g.nq2);
    prhs += int64_t(blockIdx.y) * g.nq1;
    dp += int64_t(blockIdx.y) * g.nq1;
    const int E0x = (tlin % tiles) * BT, E0y = (tlin / tiles) * BT;
    const int ox = 2 * E0x - 2, oy = 2 * E0y - 2;
    constexpr int kIt = (BQ2 * BQ2 + BNT - 1) / BNT;
    T v0[kIt], v1[kIt];
    bool f2[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int t = threadIdx.x + it * BNT;
        const int qi = ox + t % BQ2, qj = oy + t / BQ2;
        f2[it] = t < BQ2 * BQ2 && qi > 0 && qj > 0 && qi < g.s2 - 1 && qj < g.s2 - 1;
        const int64_t q = f2[it] ? int64_t(qj) * g.s2 + qi : 0;
        v0[it] = vin[q];
        v1[it] = vin[g.nq2 + q];
    }
    const int tx = threadIdx.x % BT, ty = threadIdx.x / BT;
    const int I = E0x + tx, J = E0y + ty;
    const bool node = I <= g.N && J <= g.N;
    const int64_t qp = node ? int64_t(J) * g.s1 + I : 0;
    // MODE 0 reads the pressure residual from vin, MODE 1 the stored rhs
    const T pin = MODE == 0 ? vin[2 * g.nq2 + qp] : prhs[qp];
    const T dpo = MODE == 1 ? dp[qp] : T(0);
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int t = threadIdx.x + it * BNT;
        if (t < BQ2 * BQ2) {
            const int qi = ox + t % BQ2, qj = oy + t / BQ2;
            const T di = bs_dinv<T>(g, qi & 1, qj & 1);
            s_u[0][t] = f2[it] ? di * v0[it] : T(0);
            s_u[1][t] = f2[it] ? di * v1[it] : T(0);
        }
    }
    __syncthreads();
    if (!node) return;
    const int c = (2 * ty + 2) * BQ2 + 2 * tx + 2;
    T sb = 0;
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            const int cx = st_Mq(dy) * st_G(dx), cy = st_G(dy) * st_Mq(dx);
            if (cx == 0 && cy == 0) continue;
            sb += T(cx) * s_u[0][c + dy * BQ2 + dx] + T(cy) * s_u[1][c + dy * BQ2 + dx];
        }
    const T bdu = T(-g.h / 36.0) * sb;  // (B D^{-1} vin_u) at (I, J)
    const T ds = bs_schur_diag<T>(g, I, J, inv_t);
    if (MODE == 0) {
        const T rhs = pin - inv_t * bdu;
        prhs[qp] = rhs;
        dp[qp] = wj * rhs / ds;
    } else {
        dp[qp] = dpo + wj * (pin + inv_t * bdu) / ds;
    }
}

// MODE 0: out_u = B^T dp (Dirichlet rows 0); out has 2 (2N+1)^2 values.
// MODE 1: x_u = x_u + w (1/t) D^{-1} (r_u - B^T dp), x_p = x_p + w dp, with
// x_in == nullptr meaning x_in = 0 (x_out may alias x_in).
// Batched over blockIdx.y: dp advances by g.nq1, r, x by g.n, out by 2 nq2.
template <typename T, int MODE>
__global__ __launch_bounds__(BNT) void bs_grad_kernel(Geom g, const T* dp, const T* r,
                                                      const T* xin, T* xout, T w_t, T w) {
    __shared__ T s_p[BQ1 * BQ1];
    const int tiles = (g.N + 1 + BT - 1) / BT;
    const int ntile = tiles * tiles;
    const int per_xcd = (ntile + 7) / 8;
    const int tlin = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tlin >= ntile) return;
    dp += int64_t(blockIdx.y) * g.nq1;
    if (MODE == 1) {
        r += int64_t(blockIdx.y) * g.n;
        if (xin) xin += int64_t(blockIdx.y) * g.n;
        xout += int64_t(blockIdx.y) * g.n;
    } else {
        xout += int64_t(blockIdx.y) * 2 * g.nq2;
    }
    const int E0x = (tlin % tiles) * BT, E0y = (tlin / tiles) * BT;
    constexpr int kIt = (BQ1 * BQ1 + BNT - 1) / BNT;
    T vp[kIt];
    bool f1[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int t = threadIdx.x + it * BNT;
        const int I = E0x - 1 + t % BQ1, J = E0y - 1 + t / BQ1;
        f1[it] = t < BQ1 * BQ1 && I >= 0 && J >= 0 && I <= g.N && J <= g.N;
        vp[it] = dp[f1[it] ? int64_t(J) * g.s1 + I : 0];
    }
    const int tx = threadIdx.x % BT, ty = threadIdx.x / BT;
    const int ex = E0x + tx, ey = E0y + ty;
    const bool cell = ex <= g.N && ey <= g.N;
    // this cell's Q2 nodes and the values the update reads
    int64_t qn[2][2];
    T ru[2][2][2], xu[2][2][2];
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) {
            const int i = 2 * ex + aa, j = 2 * ey + bb;
            qn[bb][aa] = (cell && i < g.s2 && j < g.s2) ? int64_t(j) * g.s2 + i : -1;
            const int64_t q = qn[bb][aa] >= 0 ? qn[bb][aa] : 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                ru[bb][aa][c] = MODE == 1 ? r[c * g.nq2 + q] : T(0);
                xu[bb][aa][c] = (MODE == 1 && xin) ? xin[c * g.nq2 + q] : T(0);
            }
        }
    const int64_t qp = cell ? int64_t(ey) * g.s1 + ex : 0;
    const T xp = (MODE == 1 && xin) ? xin[2 * g.nq2 + qp] : T(0);
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int t = threadIdx.x + it * BNT;
        if (t < BQ1 * BQ1) s_p[t] = f1[it] ? vp[it] : T(0);
    }
    __syncthreads();
    if (!cell) return;
    const int c1 = (ty + 1) * BQ1 + tx + 1;
    const T cb = T(-g.h / 36.0);
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) {
            const int64_t q = qn[bb][aa];
            if (q < 0) continue;
            const int i = 2 * ex + aa, j = 2 * ey + bb;
            const bool free = i > 0 && j > 0 && i < g.s2 - 1 && j < g.s2 - 1;
            T bx = 0, by = 0;
#pragma unroll
            for (int oy = -2; oy <= 2; ++oy) {
                if (((oy - bb) & 1) != 0) continue;
#pragma unroll
                for (int oxx = -2; oxx <= 2; ++oxx) {
                    if (((oxx - aa) & 1) != 0) continue;
                    const int cx = st_Mq(oy) * st_G(oxx);
                    const int cy = st_G(oy) * st_Mq(oxx);
                    if (cx == 0 && cy == 0) continue;
                    const T pv = s_p[c1 + ((bb - oy) / 2) * BQ1 + (aa - oxx) / 2];
                    bx += T(cx) * pv;
                    by += T(cy) * pv;
                }
            }
            const T gx = free ? cb * bx : T(0), gy = free ? cb * by : T(0);
            if (MODE == 0) {
                xout[q] = gx;
                xout[g.nq2 + q] = gy;
            } else {
                const T di = free ? bs_dinv<T>(g, aa, bb) : T(1);
                xout[q] = xu[bb][aa][0] + w_t * di * (ru[bb][aa][0] - gx);
                xout[g.nq2 + q] = xu[bb][aa][1] + w_t * di * (ru[bb][aa][1] - gy);
            }
        }
    if (MODE == 1) xout[2 * g.nq2 + qp] = xp + w * s_p[c1];
}

// ---------------------------------------------------------------------------
// Vanka update (owner computes).  A workgroup owns the elements
// [E0, E0+VT) in each direction: the Q2 nodes [2E0, 2E0+2VT) and the Q1
// nodes [E0, E0+VT).  It solves every patch that touches an owned DoF --
// the Q1 nodes [E0-1, E0+VT], VP = VT+2 = 16 per direction, one thread
// each, lanes row-major so that a row of 16 patches is one DPP row -- and
// sums the weighted corrections of each owned DoF in a fixed order, so
// every DoF is written by exactly one workgroup and the result is bitwise
// reproducible.
//
// Interior patches (distance >= 2 from the boundary) share one inverse,
// applied in the coordinates of the symmetry group of the square
// (d4_apply.h: 495 multiply-adds on compile-time constants instead of
// 2601).  The O(N) boundary patches (24 other classes) are solved first by
// vanka_boundary_kernel into a side buffer that the tile kernel reads; with
// a per-element viscosity every patch is solved that way
// (vanka_patch_kernel, one stored inverse per patch).
//
// Summation of the corrections: a patch with its lower-left window corner
// at Q2 column 2tx-4 (tile coordinates) sends slot a to column 2tx-4+a, so
// column 2m receives slot 4 of patch m, slot 2 of patch m+1 and slot 0 of
// patch m+2, and column 2m+1 slots 3 and 1 of patches m+1 and m+2.  These
// x-sums are formed with DPP row shifts inside each 16-lane row; the same
// rule in y combines rows through one LDS exchange.
// ---------------------------------------------------------------------------

constexpr int VT = 14;            // owned elements per tile side
constexpr int VP = VT + 2;        // patches per tile side (= DPP row width)
constexpr int VNT = VP * VP;      // threads per workgroup (256)
constexpr int VR = 2 * VT + 7;    // staged residual region (Q2 nodes per side)

// Interior operator: v <- D W1 D v in place for the universal interior
// operator W1 in the dihedral coordinates of symmetry.h (d4_apply.h; 495
// multiply-adds on compile-time constants) with D = diag(I, t) applied to
// the pressure output; the caller scales the input (velocity by omega/nu,
// pressure by t omega/nu with t = nu/h).
struct InteriorD4 {
    __device__ constexpr double operator()(int i) const { return kInteriorD4[i]; }
};
template <typename T>
__device__ __forceinline__ void sym_apply(T (&v)[kSlots], T t) {
    d4_apply(v, t, InteriorD4{});
}

// Keeps the compiler from carrying a value across an LDS round trip in
// registers, and the scheduler from moving any instruction across this point.
__device__ __forceinline__ void lds_order() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}
// Makes the value exist in a register at this point of the instruction
// stream (so its computation cannot sink below a following lds_order).
template <typename T>
__device__ __forceinline__ void pin(T& a) {
    asm volatile("" : "+v"(a));
}

// sym_apply with the same arithmetic in the same order, but with at most 26
// of the 51 patch values in registers at a time: the inputs of blocks 0 and 3
// wait in LDS while blocks 1 and 2 are formed, and the outputs of blocks 1
// and 2 while blocks 0 and 3 are.  `park` is this lane's column of a
// [26][VNT] LDS area that no other lane touches.
constexpr int kPark = 26;
template <typename T>
__device__ __forceinline__ void sym_apply_parked(T (&v)[kSlots], T t, T* park) {
    const D4Table& d = kD4Table;
    const InteriorD4 coef{};
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int b = 0; b < 5; ++b) d4_bfly(v, 25 * f + 5 * b, 1);
#pragma unroll
        for (int q = 0; q < 5; ++q) d4_bfly(v, 25 * f + q, 5);
    }
    // inputs of blocks 0 (pressure, pairs a0/b0) and 3 (pairs a3/b3)
    park[0] = v[50];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        park[(1 + k) * VNT] = v[d.a0[k]];
        park[(7 + k) * VNT] = v[d.b0[k]];
        park[(13 + k) * VNT] = v[d.a3[k]];
        park[(19 + k) * VNT] = v[d.b3[k]];
    }
    lds_order();
    // blocks 1 and 2: one set of constants, each used twice
    T y1[13], y2[13];
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        T a1 = 0, a2 = 0;
#pragma unroll
        for (int k = 0; k < 13; ++k) {
            const T c = T(coef(kD4Off1 + i * 13 + k));
            a1 += c * v[d.m1[k]];
            a2 += c * v[d.m2[k]];
        }
        y1[i] = a1;
        y2[i] = a2;
    }
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        pin(y1[i]);
        pin(y2[i]);
    }
    lds_order();
    v[50] = park[0];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        v[d.a0[k]] = park[(1 + k) * VNT];
        v[d.b0[k]] = park[(7 + k) * VNT];
        v[d.a3[k]] = park[(13 + k) * VNT];
        v[d.b3[k]] = park[(19 + k) * VNT];
    }
    lds_order();
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        park[i * VNT] = y1[i];
        park[(13 + i) * VNT] = y2[i];
    }
    lds_order();
    // block 0: even (p and pair sums) and odd (pair differences) parts
    {
        T e[7], o[6], ye[7], yo[6];
        e[0] = v[50];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            e[k + 1] = v[d.a0[k]] + v[d.b0[k]];
            o[k] = v[d.a0[k]] - v[d.b0[k]];
        }
        d4_block(e, ye, kD4Off0e, coef);
        d4_block(o, yo, kD4Off0o, coef);
        v[50] = ye[0];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            v[d.a0[k]] = ye[k + 1] + yo[k];
            v[d.b0[k]] = ye[k + 1] - yo[k];
        }
    }
    // block 3: pair sums and differences
    {
        T e[6], o[6], ye[6], yo[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            e[k] = v[d.a3[k]] + v[d.b3[k]];
            o[k] = v[d.a3[k]] - v[d.b3[k]];
        }
        d4_block(e, ye, kD4Off3e, coef);
        d4_block(o, yo, kD4Off3o, coef);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            v[d.a3[k]] = ye[k] + yo[k];
            v[d.b3[k]] = ye[k] - yo[k];
        }
    }
    v[50] *= t;
    pin(v[50]);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        pin(v[d.a0[k]]);
        pin(v[d.b0[k]]);
        pin(v[d.a3[k]]);
        pin(v[d.b3[k]]);
    }
    lds_order();
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        v[d.m1[i]] = park[i * VNT];
        v[d.m2[i]] = park[(13 + i) * VNT];
    }
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int q = 0; q < 5; ++q) d4_bfly_t(v, 25 * f + q, 5);
#pragma unroll
        for (int b = 0; b < 5; ++b) d4_bfly_t(v, 25 * f + 5 * b, 1);
    }
}

// Value of lane (l + S) of the same 16-lane row, 0 past the row end
// (DPP row_shl; the 64-bit value moves as two 32-bit halves).
template <int S>
__device__ __forceinline__ double row_shl(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(u & 0xffffffffLL), 0x100 + S, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, int(u >> 32), 0x100 + S, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<unsigned int>(lo));
}
template <int S>
__device__ __forceinline__ float row_shl(float v) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + S, 0xF, 0xF, true));
}

__device__ __forceinline__ int dclass(int i, int N) {
    return i == 0 ? 0 : i == N ? 4 : i == 1 ? 1 : i == N - 1 ? 3 : 2;
}

// Boundary patches (Q1 nodes within one element of the boundary, 8N - 8 of
// them, N >= 4) in an order that groups patches of one class: rows 0, 1,
// N-1, N in full, then the columns 0, 1, N-1, N of the rows 2..N-2, one
// column after the other (each such column is a single class).
__host__ __device__ inline int n_boundary_patches(int N) { return 8 * N - 8; }

__device__ __forceinline__ void boundary_patch(int k, int N, int& I, int& J) {
    const int w = N + 1;
    if (k < 4 * w) {
        const int rrow = k / w;
        J = rrow < 2 ? rrow : N - 3 + rrow;
        I = k % w;
    } else {
        k -= 4 * w;
        const int c = k / (N - 3);
        J = 2 + k % (N - 3);
        I = c < 2 ? c : N - 3 + c;
    }
}

__device__ __forceinline__ int boundary_index(int I, int J, int N) {
    const int w = N + 1;
    if (J <= 1) return J * w + I;
    if (J >= N - 1) return (J - N + 3) * w + I;
    const int c = I <= 1 ? I : I - N + 3;
    return 4 * w + c * (N - 3) + (J - 2);
}

// Global index of patch slot s of the patch at Q1 node (I, J), or -1 if the
// slot lies outside the domain.
__device__ __forceinline__ int64_t slot_index(const Geom& g, int I, int J, int s) {
    if (s == 50) return 2 * g.nq2 + int64_t(J) * g.s1 + I;
    const int f = s / 25, l = s % 25;
    const int qi = 2 * I - 2 + l % 5, qj = 2 * J - 2 + l / 5;
    if (qi < 0 || qj < 0 || qi >= g.s2 || qj >= g.s2) return -1;
    return int64_t(f) * g.nq2 + int64_t(qj) * g.s2 + qi;
}

// Boundary patches, KBP consecutive ones (in the class-grouped order) per
// wavefront: lane s gathers slot s of every patch, then computes row s of
// the class's weighted inverse (stored transposed, so the lanes read
// consecutive addresses) against each patch residual broadcast from LDS.
// The coefficient row stays in registers while the class does not change,
// so a wavefront usually loads it once for all its patches.  Gathers and
// the first class's coefficients are issued together (inactive lanes read
// valid addresses and are discarded).  Several patches per wavefront cut
// the coefficient traffic (51 x 51 values per patch otherwise) on the large
// levels; one per wavefront keeps the dependent chain short on the small
// ones (boundary_patches_per_wave).
template <typename T, int KBP>
__global__ __launch_bounds__(256) void vanka_boundary_kernel(Geom g, const T* __restrict__ rb,
                                                             const T* __restrict__ table,
                                                             T* __restrict__ dbuf) {
    constexpr int kBP = KBP;
    __shared__ T s_r[4][kBP][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nb = n_boundary_patches(g.N);
    rb += int64_t(blockIdx.y) * g.n;  // right-hand side blockIdx.y of a batch
    dbuf += int64_t(blockIdx.y) * nb * 64;
    const int k0 = (blockIdx.x * 4 + w) * kBP;
    const int s = lane < kSlots ? lane : 0;
    int cls[kBP];
    T rv[kBP];
    bool ok[kBP];
#pragma unroll
    for (int p = 0; p < kBP; ++p) {
        int I = 0, J = 0;
        const bool active = k0 + p < nb;
        if (active) boundary_patch(k0 + p, g.N, I, J);
        cls[p] = 5 * dclass(J, g.N) + dclass(I, g.N);
        const int64_t q = slot_index(g, I, J, s);
        ok[p] = active && lane < kSlots && q >= 0;
        rv[p] = rb[q >= 0 ? q : 0];
    }
    T m[kSlots];
    int cur = cls[0];
#pragma unroll
    for (int t = 0; t < kSlots; ++t) m[t] = table[(cur * kSlots + t) * kSlots + s];
#pragma unroll
    for (int p = 0; p < kBP; ++p) s_r[w][p][lane] = ok[p] ? rv[p] : T(0);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kBP; ++p) {
        if (k0 + p >= nb) break;
        if (cls[p] != cur) {  // uniform over the wavefront
            cur = cls[p];
#pragma unroll
            for (int t = 0; t < kSlots; ++t) m[t] = table[(cur * kSlots + t) * kSlots + s];
        }
        T a0 = 0, a1 = 0;
#pragma unroll
        for (int t = 0; t + 1 < kSlots; t += 2) {
            a0 += m[t] * s_r[w][p][t];
            a1 += m[t + 1] * s_r[w][p][t + 1];
        }
        a0 += m[kSlots - 1] * s_r[w][p][kSlots - 1];
        if (lane < kSlots) dbuf[int64_t(k0 + p) * 64 + lane] = a0 + a1;
    }
}

// "Simple" Vanka for a per-element viscosity: every patch has its own
// stored weighted inverse (transposed, 51 x 51 per patch, patch k =
// J*(N+1) + I); one wavefront per patch, lane s computing correction slot s
// (column reads coalesced over the lanes) into dbuf[k*64 + s].  Batched over
// blockIdx.y (rb by g.n, dbuf by (N+1)^2 * 64); the tables are shared.
template <typename T>
__global__ __launch_bounds__(256) void vanka_patch_kernel(Geom g, const T* __restrict__ rb,
                                                          const T* __restrict__ tables,
                                                          T* __restrict__ dbuf) {
    __shared__ T s_r[4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int np = (g.N + 1) * (g.N + 1);
    rb += int64_t(blockIdx.y) * g.n;
    dbuf += int64_t(blockIdx.y) * np * 64;
    const int k = blockIdx.x * 4 + w;
    const bool active = k < np;
    const int kk = active ? k : 0;
    const int I = kk % (g.N + 1), J = kk / (g.N + 1);
    const int s = lane < kSlots ? lane : 0;
    const int64_t q = slot_index(g, I, J, s);
    const T rv = rb[q >= 0 ? q : 0];
    const T* tb = tables + int64_t(kk) * kSlots * kSlots;
    T m[kSlots];
#pragma unroll
    for (int t = 0; t < kSlots; ++t) m[t] = tb[t * kSlots + s];
    s_r[w][lane] = (active && lane < kSlots && q >= 0) ? rv : T(0);
    __syncthreads();
    T a0 = 0, a1 = 0;
#pragma unroll
    for (int t = 0; t + 1 < kSlots; t += 2) {
        a0 += m[t] * s_r[w][t];
        a1 += m[t + 1] * s_r[w][t + 1];
    }
    a0 += m[kSlots - 1] * s_r[w][kSlots - 1];
    if (active && lane < kSlots) dbuf[int64_t(k) * 64 + lane] = a0 + a1;
}

// Tile grid and the XCD-aware tile order: consecutive workgroup ids are
// dealt round-robin to the 8 XCDs, so id L takes tile (L mod 8) ceil(T/8) +
// L/8 in row-major order, giving every XCD a contiguous band of tiles whose
// shared halos stay in its L2.
__host__ __device__ inline int vanka_tiles(int N) { return (N + 1 + VT - 1) / VT; }

// Staged region of the sweep kernel (per tile, Q2 / Q1 nodes per side):
//   r region: Q2 [2E0-4, 2E0+2VT+2], Q1 [E0-1, E0+VT]
constexpr int VR1 = VT + 2;
// The staged residual of a component (VR x VR Q2 nodes) is stored by column
// parity, even columns then odd ones, each half with row stride VRS: the
// gather reads column 2tx + a, so the 16 lanes of a patch row then read
// consecutive words, and with VRS = 24 the four patch rows of a wavefront
// (two node rows apart) start 32 words apart (no LDS bank conflicts; the
// plain row-major layout has the lanes of a row two words apart).
constexpr int VRS = 24;
constexpr int kRHalf = VR * VRS;
constexpr int kRComp = 2 * kRHalf;
__host__ __device__ constexpr int rr_at(int row, int col) {
    return (col & 1) * kRHalf + row * VRS + (col >> 1);
}
static_assert((VR + 1) / 2 <= VRS, "a column-parity half fits its row stride");
constexpr int kRRegion = 2 * kRComp + VR1 * VR1;
constexpr int kExchange = 20 * VNT;
constexpr int kSweepLds = (kRRegion > kExchange) ? kRRegion : kExchange;
constexpr int kSweepLdsPark = (kSweepLds > kPark * VNT) ? kSweepLds : kPark * VNT;

// Stage the scaled residual of a tile's r region in LDS (velocity scaled
// by `scale`, pressure by `scale * t`, nodes outside the mesh zero).  All
// global loads are issued before the first is used.
template <typename T>
__device__ __forceinline__ void stage_residual_region(const Geom& g, const T* __restrict__ rb,
                                                      int E0x, int E0y, T scale, T t,
                                                      T* __restrict__ sr0, T* __restrict__ sr1,
                                                      T* __restrict__ srp) {
    constexpr int kIt = (VR * VR + VNT - 1) / VNT;
    const int ox = 2 * E0x - 4, oy = 2 * E0y - 4;
    T v0[kIt], v1[kIt];
    bool in[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int k = threadIdx.x + it * VNT;
        const int qi = ox + k % VR, qj = oy + k / VR;
        in[it] = k < VR * VR && qi >= 0 && qj >= 0 && qi < g.s2 && qj < g.s2;
        const int64_t q = in[it] ? int64_t(qj) * g.s2 + qi : 0;
        v0[it] = rb[q];
        v1[it] = rb[g.nq2 + q];
    }
    const int I = E0x - 1 + threadIdx.x % VP, J = E0y - 1 + threadIdx.x / VP;
    const bool valid = I >= 0 && J >= 0 && I <= g.N && J <= g.N;
    const T vp = rb[2 * g.nq2 + (valid ? int64_t(J) * g.s1 + I : 0)];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int k = threadIdx.x + it * VNT;
        if (k < VR * VR) {
            const int l = rr_at(k / VR, k % VR);
            sr0[l] = in[it] ? scale * v0[it] : T(0);
            sr1[l] = in[it] ? scale * v1[it] : T(0);
        }
    }
    srp[threadIdx.x] = valid ? (scale * t) * vp : T(0);
}

// Owner update of a tile from the LDS row sums xs (entry e = (b*2 + c)*2 +
// parity at xs[e * VNT + patch]): thread (tx, ty) < VT owns the Q2 nodes
// (2E0+2tx+px, 2E0+2ty+py); Dirichlet nodes keep x_in.  Loads first.
template <typename T>
__device__ __forceinline__ void owner_update_velocity(const Geom& g, const T* __restrict__ xs,
                                                      int E0x, int E0y, const T* xin, T* xout) {
    const int tx = threadIdx.x % VP, ty = threadIdx.x / VP;
    if (tx >= VT || ty >= VT) return;
    const int gi0 = 2 * E0x + 2 * tx, gj0 = 2 * E0y + 2 * ty;
    int64_t qn[2][2][2];
    T base[2][2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int px = 0; px < 2; ++px)
#pragma unroll
            for (int py = 0; py < 2; ++py) {
                const int gi = gi0 + px, gj = gj0 + py;
                const bool in = gi < g.s2 && gj < g.s2;
                qn[c][px][py] = in ? int64_t(c) * g.nq2 + int64_t(gj) * g.s2 + gi : -1;
                base[c][px][py] = xin ? xin[in ? qn[c][px][py] : 0] : T(0);
            }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int px = 0; px < 2; ++px) {
            auto at = [&](int b, int dty) {
                return xs[((b * 2 + c) * 2 + px) * VNT + threadIdx.x + dty * VP];
            };
            const T even_row = at(4, 0) + at(2, 1) + at(0, 2);
            const T odd_row = at(3, 1) + at(1, 2);
            const int gi = gi0 + px;
#pragma unroll
            for (int py = 0; py < 2; ++py) {
                const int gj = gj0 + py;
                if (qn[c][px][py] < 0) continue;
                const bool free = gi > 0 && gj > 0 && gi < g.s2 - 1 && gj < g.s2 - 1;
                xout[qn[c][px][py]] = free ? base[c][px][py] + (py ? odd_row : even_row)
                                           : base[c][px][py];
            }
        }
}

// The same update with its loads issued early: owner_prefetch at the start
// of the kernel (the loads are in flight during the patch solves; DoFs are
// owned by one workgroup, so reading x_in first is safe in place too), then
// owner_commit after the exchange.
template <typename T>
struct OwnerBase {
    T v[2][2][2];
    T p;
};

template <typename T>
__device__ __forceinline__ void owner_prefetch(const Geom& g, int E0x, int E0y, const T* xin,
                                               OwnerBase<T>& ob) {
    const int tx = threadIdx.x % VP, ty = threadIdx.x / VP;
    const bool own = tx < VT && ty < VT;
    const int gi0 = 2 * E0x + 2 * tx, gj0 = 2 * E0y + 2 * ty;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int px = 0; px < 2; ++px)
#pragma unroll
            for (int py = 0; py < 2; ++py) {
                const int gi = gi0 + px, gj = gj0 + py;
                const bool in = own && gi < g.s2 && gj < g.s2;
                const int64_t q = in ? int64_t(c) * g.nq2 + int64_t(gj) * g.s2 + gi : 0;
                ob.v[c][px][py] = xin ? xin[q] : T(0);
            }
    // owned pressure: Q1 node (E0 - 1 + tx, E0 - 1 + ty) for 1 <= tx, ty <= VT
    const int I = E0x - 1 + tx, J = E0y - 1 + ty;
    const bool pin = tx >= 1 && ty >= 1 && tx <= VT && ty <= VT && I <= g.N && J <= g.N;
    ob.p = xin ? xin[2 * g.nq2 + (pin ? int64_t(J) * g.s1 + I : 0)] : T(0);
}

template <typename T>
__device__ __forceinline__ void owner_commit(const Geom& g, const T* __restrict__ xs, int E0x,
                                             int E0y, const OwnerBase<T>& ob, T* xout) {
    const int tx = threadIdx.x % VP, ty = threadIdx.x / VP;
    if (tx >= VT || ty >= VT) return;
    const int gi0 = 2 * E0x + 2 * tx, gj0 = 2 * E0y + 2 * ty;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int px = 0; px < 2; ++px) {
            auto at = [&](int b, int dty) {
                return xs[((b * 2 + c) * 2 + px) * VNT + threadIdx.x + dty * VP];
            };
            const T even_row = at(4, 0) + at(2, 1) + at(0, 2);
            const T odd_row = at(3, 1) + at(1, 2);
            const int gi = gi0 + px;
#pragma unroll
            for (int py = 0; py < 2; ++py) {
                const int gj = gj0 + py;
                if (gi >= g.s2 || gj >= g.s2) continue;
                const int64_t q = int64_t(c) * g.nq2 + int64_t(gj) * g.s2 + gi;
                const bool free = gi > 0 && gj > 0 && gi < g.s2 - 1 && gj < g.s2 - 1;
                xout[q] = free ? ob.v[c][px][py] + (py ? odd_row : even_row) : ob.v[c][px][py];
            }
        }
}

// One additive Vanka sweep on a tile given the residual r (`rb`) of x_in:
// x_out = x_in + corrections, with x_in == x_out allowed (in place) and
// x_in == nullptr meaning x_in = 0.  Every DoF a tile owns is written
// (Dirichlet DoFs keep x_in).  The interior operator is applied to the
// residual scaled by omega/nu (pressure also by t = nu/h), see sym_apply.
// SIMPLE: every patch correction comes from dbuf (vanka_patch_kernel, patch
// k = J*(N+1) + I) instead of the interior operator and the boundary kernel.
// PARK: the interior operator through sym_apply_parked (same results), for
// three waves per SIMD instead of two.
template <typename T, bool SIMPLE = false, bool PARK = false>
__global__ __launch_bounds__(VNT, PARK ? 3 : 2) void vanka_sweep_kernel(Geom g, const T* __restrict__ rb,
                                                             const T* xin, T* xout,
                                                             const T* __restrict__ dbuf, T scale,
                                                             T t) {
    __shared__ T s_buf[PARK ? kSweepLdsPark : kSweepLds];
    T* const sr0 = s_buf;
    T* const sr1 = sr0 + kRComp;
    T* const srp = sr1 + kRComp;
    const int tiles = vanka_tiles(g.N);
    const int ntile = tiles * tiles;
    const int per_xcd = (ntile + 7) / 8;
    const int tlin = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tlin >= ntile) return;
    {  // right-hand side blockIdx.y of a batch
        const int64_t bo = int64_t(blockIdx.y) * g.n;
        rb += bo;
        if (xin) xin += bo;
        xout += bo;
        dbuf += int64_t(blockIdx.y) * (SIMPLE ? (g.N + 1) * (g.N + 1) : n_boundary_patches(g.N)) * 64;
    }
    const int E0x = (tlin % tiles) * VT, E0y = (tlin / tiles) * VT;
    // the owners' x loads are issued here and land while the patches are
    // solved (the boundary-patch index below is formed before the staging:
    // with it formed after the apply, the parked form had no registers left
    // for these loads)
    OwnerBase<T> ob;
    owner_prefetch(g, E0x, E0y, xin, ob);
    const int tx = threadIdx.x % VP, ty = threadIdx.x / VP;
    const int I = E0x - 1 + tx, J = E0y - 1 + ty;
    const bool valid = I >= 0 && J >= 0 && I <= g.N && J <= g.N;

    T rv[kSlots];
    if (SIMPLE) {
        const int64_t bi = valid ? int64_t(J) * (g.N + 1) + I : 0;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) rv[s] = valid ? dbuf[bi * 64 + s] : T(0);
    } else {
        const bool interior = valid && I >= 2 && J >= 2 && I <= g.N - 2 && J <= g.N - 2;
        const int bi = valid && !interior ? boundary_index(I, J, g.N) : 0;
        stage_residual_region(g, rb, E0x, E0y, scale, t, sr0, sr1, srp);
        __syncthreads();
#pragma unroll
        for (int b = 0; b < 5; ++b)
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                const int l = rr_at(2 * ty + b, 2 * tx + a);
                rv[5 * b + a] = sr0[l];
                rv[25 + 5 * b + a] = sr1[l];
            }
        rv[50] = srp[ty * VR1 + tx];

        if (PARK) {
            __syncthreads();  // the park area overlaps the staged residual
            sym_apply_parked(rv, t, s_buf + threadIdx.x);
        } else {
            sym_apply(rv, t);  // interior operator, every lane
        }
        if (!interior) {
            // boundary patch: corrections precomputed; outside the domain: none
#pragma unroll
            for (int s = 0; s < kSlots; ++s) rv[s] = valid ? dbuf[int64_t(bi) * 64 + s] : T(0);
        }
    }
    __syncthreads();  // the staging buffers are reused for the exchange below

    // x-sums within the 16-lane rows: column 2tx (even) and 2tx+1 (odd) of
    // patch row slot b, both components; exchanged through LDS by b
    T* xs = s_buf;  // 20 values per thread: [(b*2 + c)*2 + parity][thread]
#pragma unroll
    for (int b = 0; b < 5; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int o = 25 * c + 5 * b;
            const T ev = rv[o + 4] + row_shl<1>(rv[o + 2]) + row_shl<2>(rv[o + 0]);
            const T od = row_shl<1>(rv[o + 3]) + row_shl<2>(rv[o + 1]);
            const int base = ((b * 2 + c) * 2) * VNT;
            xs[base + threadIdx.x] = ev;
            xs[base + VNT + threadIdx.x] = od;
        }
    __syncthreads();
    owner_commit(g, xs, E0x, E0y, ob, xout);
    if (valid && tx >= 1 && tx <= VT && ty >= 1 && ty <= VT) {
        const int64_t q = 2 * g.nq2 + int64_t(J) * g.s1 + I;
        xout[q] = ob.p + rv[50];
    }
}

// ---------------------------------------------------------------------------
// Fused sweep for the small levels (latency-bound there): r = b - A x_in
// and the Vanka update x_out = x_in + sum_i V_i^T W_i A_i^{-1} V_i r in ONE
// launch, instead of the residual, boundary-patch and tile launches.  Same
// tile, patch order and owner sums as vanka_sweep_kernel, and the same
// arithmetic in the same order as those three kernels (results bitwise
// equal), with x_out != x_in (a tile reads x_in up to three elements beyond
// the DoFs it owns).  XIN = false: x_in = 0, so r = b.
//
// Workgroup of 12 waves:
//   * all waves stage x_in (Q2 nodes [2E0-6, 2E0+2VT+6), Q1 [E0-3, E0+VT+3),
//     Dirichlet and outside nodes zero, as residual_kernel) and then form
//     the residual of the tile's r region (18 x 18 cells, two row parities:
//     cell_row_pair on the staged values) into LDS, unscaled;
//   * waves 0-3: one patch per lane as in vanka_sweep_kernel (gather with
//     the scaling of stage_residual_region, interior operator, owner sums);
//   * waves 4-11: the tile's boundary patches row-parallel, as
//     vanka_boundary_kernel, one class per wave so that its coefficient rows
//     are loaded once, during the staging: waves 4/5 the non-corner patches
//     of the (at most two) boundary patch rows of the tile, 6/7 those of the
//     boundary patch columns, 8-11 the (at most four) corner patches.  Their
//     corrections go to an LDS slot table that the boundary lanes of waves
//     0-3 read before the owner sums.
// Needs N >= 16 (a tile then meets at most two boundary patch rows and two
// boundary patch columns).
// ---------------------------------------------------------------------------

constexpr int FX2 = 2 * VT + 12;  // staged Q2 nodes of x_in per side (offset -6)
constexpr int FX1 = VT + 6;       // staged Q1 nodes of x_in per side (offset -3)
constexpr int FC = VT + 4;        // cells per side whose rows are formed (offset -2)
constexpr int FNT = 3 * VNT;      // threads per workgroup
constexpr int kFItems = 2 * FC * FC;                     // (cell, row parity) items
constexpr int kFX = 2 * FX2 * FX2 + FX1 * FX1;           // staged x_in
constexpr int kFSlots = 68;                              // rows 0-31, columns 32-63, corners 64-67
constexpr int kFSlotStride = 52;
constexpr int kFArea = (kPark * VNT > kFX) ? kPark * VNT : kFX;  // x_in, then park, then exchange
constexpr int kFusedLds = kFArea + kRRegion + kFSlots * kFSlotStride;
constexpr int kFusedMinN = 16;
static_assert(kFItems <= FNT, "one residual item per thread");
static_assert(kExchange <= kFArea, "exchange fits the staging area");

// The boundary patch rows (J) or columns (I) that a tile window
// [E0 - 1, E0 + VP - 2] meets, in increasing order: at most two for N >= 16.
__device__ __forceinline__ int tile_boundary_lines(int E0, int N, int (&line)[2]) {
    const int cand[4] = {0, 1, N - 1, N};
    int k = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int v = cand[c];
        if (v >= E0 - 1 && v <= E0 + VP - 2 && k < 2) line[k++] = v;
    }
    if (k < 2) line[1] = -1;
    if (k < 1) line[0] = -1;
    return k;
}

template <typename T, bool XIN>
__global__ __launch_bounds__(FNT, 1) void vanka_fused_kernel(Geom g, const T* __restrict__ b,
                                                             const T* __restrict__ xin,
                                                             T* __restrict__ xout,
                                                             const T* __restrict__ table,
                                                             T scale, T t) {
    constexpr bool kPark = std::is_same<T, double>::value;  // FP64: parked interior apply
    __shared__ T s_buf[kFusedLds];
    T* const sx0 = s_buf;                 // staged x_in (phase 1)
    T* const sx1 = sx0 + FX2 * FX2;
    T* const sxp = sx1 + FX2 * FX2;
    T* const sr0 = s_buf + kFArea;        // residual of the r region (unscaled)
    T* const sr1 = sr0 + kRComp;
    T* const srp = sr1 + kRComp;
    T* const sdel = sr0 + kRRegion;       // boundary-patch corrections by slot
    const int tiles = vanka_tiles(g.N);
    const int ntile = tiles * tiles;
    const int per_xcd = (ntile + 7) / 8;
    const int tlin = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tlin >= ntile) return;
    {  // right-hand side blockIdx.y of a batch
        const int64_t bo = int64_t(blockIdx.y) * g.n;
        b += bo;
        if (XIN) xin += bo;
        xout += bo;
    }
    const int E0x = (tlin % tiles) * VT, E0y = (tlin / tiles) * VT;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    int brow[2], bcol[2];
    const int nbr = tile_boundary_lines(E0y, g.N, brow);
    const int nbc = tile_boundary_lines(E0x, g.N, bcol);

    // ---- phase 0: every global load of the staging is issued first (the
    // owners' x_in loads too, except with the parked apply, which has no
    // registers to spare for them: there they follow the apply)
    OwnerBase<T> ob;
    if (!kPark && wave < 4) owner_prefetch(g, E0x, E0y, XIN ? xin : nullptr, ob);

    // boundary waves: their group (class) and its coefficient rows
    const int bw = wave - 4;
    int gcls = -1;
    if (bw >= 0) {
        if (bw < 2) {
            if (bw < nbr) gcls = 5 * dclass(brow[bw], g.N) + 2;
        } else if (bw < 4) {
            if (bw - 2 < nbc) gcls = 10 + dclass(bcol[bw - 2], g.N);
        } else {
            const int rr = (bw - 4) >> 1, cc = (bw - 4) & 1;
            if (rr < nbr && cc < nbc) gcls = 5 * dclass(brow[rr], g.N) + dclass(bcol[cc], g.N);
        }
    }
    // (loaded with the staging when no residual is formed, else once this
    // thread's residual item is done: registers)
    const int cs = lane < kSlots ? lane : 0;
    T m[kSlots];
    if (!XIN && gcls >= 0) {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) m[k] = table[(gcls * kSlots + k) * kSlots + cs];
    }

    // residual item of this thread: cell (ex, ey), row parity bb
    const int item = tid;
    const bool has_item = XIN && item < kFItems;
    const int bb = (item / (FC * FC)) & 1;
    const int cidx = item % (FC * FC);
    const int cx = cidx % FC, cy = cidx / FC;
    const int ex = E0x - 2 + cx, ey = E0y - 2 + cy;
    int64_t qn[2];
    bool inm[2], dir[2];
    T bxv[2], byv[2], xdx[2], xdy[2];
    T bp = 0;
    const bool pitem = has_item && bb == 0 && cx >= 1 && cx <= VT + 2 && cy >= 1 && cy <= VT + 2;
    const bool pin = pitem && ex >= 0 && ey >= 0 && ex <= g.N && ey <= g.N;
    if (XIN) {
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) {
            const int i = 2 * ex + aa, j = 2 * ey + bb;
            inm[aa] = has_item && i >= 0 && j >= 0 && i < g.s2 && j < g.s2;
            dir[aa] = inm[aa] && (i == 0 || j == 0 || i == g.s2 - 1 || j == g.s2 - 1);
            qn[aa] = inm[aa] ? int64_t(j) * g.s2 + i : 0;
            bxv[aa] = b[qn[aa]];
            byv[aa] = b[g.nq2 + qn[aa]];
            xdx[aa] = xin[qn[aa]];
            xdy[aa] = xin[g.nq2 + qn[aa]];
        }
        bp = b[2 * g.nq2 + (pin ? int64_t(ey) * g.s1 + ex : 0)];

        // x_in on the staged nodes (clamped addresses, zeroed afterwards)
        constexpr int kI2 = (FX2 * FX2 + FNT - 1) / FNT, kI1 = (FX1 * FX1 + FNT - 1) / FNT;
        T v0[kI2], v1[kI2], vp[kI1];
        bool f2[kI2], f1[kI1];
        const int ox = 2 * E0x - 6, oy = 2 * E0y - 6;
#pragma unroll
        for (int it = 0; it < kI2; ++it) {
            const int k = tid + it * FNT;
            const int qi = ox + k % FX2, qj = oy + k / FX2;
            f2[it] = k < FX2 * FX2 && qi > 0 && qj > 0 && qi < g.s2 - 1 && qj < g.s2 - 1;
            const int64_t q = f2[it] ? int64_t(qj) * g.s2 + qi : 0;
            v0[it] = xin[q];
            v1[it] = xin[g.nq2 + q];
        }
#pragma unroll
        for (int it = 0; it < kI1; ++it) {
            const int k = tid + it * FNT;
            const int I = E0x - 3 + k % FX1, J = E0y - 3 + k / FX1;
            f1[it] = k < FX1 * FX1 && I >= 0 && J >= 0 && I <= g.N && J <= g.N;
            vp[it] = xin[2 * g.nq2 + (f1[it] ? int64_t(J) * g.s1 + I : 0)];
        }
#pragma unroll
        for (int it = 0; it < kI2; ++it) {
            const int k = tid + it * FNT;
            if (k < FX2 * FX2) {
                sx0[k] = f2[it] ? v0[it] : T(0);
                sx1[k] = f2[it] ? v1[it] : T(0);
            }
        }
#pragma unroll
        for (int it = 0; it < kI1; ++it) {
            const int k = tid + it * FNT;
            if (k < FX1 * FX1) sxp[k] = f1[it] ? vp[it] : T(0);
        }
    } else {
        // r = b on the r region (nodes outside the mesh zero)
        constexpr int kIt = (VR * VR + FNT - 1) / FNT;
        const int ox = 2 * E0x - 4, oy = 2 * E0y - 4;
        T v0[kIt], v1[kIt];
        bool in[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int k = tid + it * FNT;
            const int qi = ox + k % VR, qj = oy + k / VR;
            in[it] = k < VR * VR && qi >= 0 && qj >= 0 && qi < g.s2 && qj < g.s2;
            const int64_t q = in[it] ? int64_t(qj) * g.s2 + qi : 0;
            v0[it] = b[q];
            v1[it] = b[g.nq2 + q];
        }
        const int I = E0x - 1 + tid % VR1, J = E0y - 1 + tid / VR1;
        const bool pv = tid < VR1 * VR1 && I >= 0 && J >= 0 && I <= g.N && J <= g.N;
        const T vpp = b[2 * g.nq2 + (pv ? int64_t(J) * g.s1 + I : 0)];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int k = tid + it * FNT;
            if (k < VR * VR) {
                const int l = rr_at(k / VR, k % VR);
                sr0[l] = in[it] ? v0[it] : T(0);
                sr1[l] = in[it] ? v1[it] : T(0);
            }
        }
        if (tid < VR1 * VR1) srp[tid] = pv ? vpp : T(0);
    }
    __syncthreads();

    // ---- phase 1: residual rows of the r region (cell_row_pair, as residual_kernel)
    if (XIN && has_item) {
        T ax[2], ay[2], ap;
        const int c2 = (2 * cy + 2) * FX2 + 2 * cx + 2, c1 = (cy + 1) * FX1 + cx + 1;
        const T cl = T(g.nu / 90.0), cb = T(-g.h / 36.0);
        if (bb == 0)
            cell_row_pair<FX2, FX1, 0>(sx0, sx1, sxp, c2, c1, cl, cb, ax, ay, ap);
        else
            cell_row_pair<FX2, FX1, 1>(sx0, sx1, sxp, c2, c1, cl, cb, ax, ay, ap);
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) {
            const int rx = 2 * cx + aa, ry = 2 * cy + bb;
            if (rx >= VR || ry >= VR) continue;
            const T vx = dir[aa] ? xdx[aa] : ax[aa];
            const T vy = dir[aa] ? xdy[aa] : ay[aa];
            sr0[rr_at(ry, rx)] = inm[aa] ? bxv[aa] - vx : T(0);
            sr1[rr_at(ry, rx)] = inm[aa] ? byv[aa] - vy : T(0);
        }
        if (pitem) srp[(cy - 1) * VR1 + cx - 1] = pin ? bp - ap : T(0);
    }
    if (XIN) {
        if (gcls >= 0) {
#pragma unroll
            for (int k = 0; k < kSlots; ++k) m[k] = table[(gcls * kSlots + k) * kSlots + cs];
        }
        __syncthreads();
    }

    // ---- phase 2: patch solves
    const int tx = tid % VP, ty = (tid / VP) % VP;
    const int I = E0x - 1 + tx, J = E0y - 1 + ty;
    const bool valid = I >= 0 && J >= 0 && I <= g.N && J <= g.N;
    T rv[kSlots];
    if (wave < 4) {
#pragma unroll
        for (int bq = 0; bq < 5; ++bq)
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                const int l = rr_at(2 * ty + bq, 2 * tx + a);
                rv[5 * bq + a] = scale * sr0[l];
                rv[25 + 5 * bq + a] = scale * sr1[l];
            }
        rv[50] = (scale * t) * srp[ty * VR1 + tx];
        if (kPark)
            sym_apply_parked(rv, t, s_buf + tid);
        else
            sym_apply(rv, t);
    } else if (gcls >= 0) {
        // this wave's boundary patches: position p of its row, column or corner
        const int np = bw < 4 ? VP : 1;
        for (int p = 0; p < np; ++p) {
            int px, py, slot;
            if (bw < 2) {
                px = p;
                py = brow[bw] - E0y + 1;
                slot = bw * VP + p;
            } else if (bw < 4) {
                px = bcol[bw - 2] - E0x + 1;
                py = p;
                slot = 2 * VP + (bw - 2) * VP + p;
            } else {
                px = bcol[(bw - 4) & 1] - E0x + 1;
                py = brow[(bw - 4) >> 1] - E0y + 1;
                slot = 4 * VP + (bw - 4);
            }
            const int pI = E0x - 1 + px, pJ = E0y - 1 + py;
            const bool mid_i = pI >= 2 && pI <= g.N - 2, mid_j = pJ >= 2 && pJ <= g.N - 2;
            const bool take = pI >= 0 && pI <= g.N && pJ >= 0 && pJ <= g.N &&
                              (bw < 2 ? mid_i : bw < 4 ? mid_j : true);
            if (!take) continue;  // uniform over the wave
            auto rs = [&](int s) -> T {
                if (s == kSlots - 1) return srp[py * VR1 + px];
                const int f = s / 25, l = s % 25;
                return (f ? sr1 : sr0)[rr_at(2 * py + l / 5, 2 * px + l % 5)];
            };
            T a0 = 0, a1 = 0;
#pragma unroll
            for (int k = 0; k + 1 < kSlots; k += 2) {
                a0 += m[k] * rs(k);
                a1 += m[k + 1] * rs(k + 1);
            }
            a0 += m[kSlots - 1] * rs(kSlots - 1);
            if (lane < kSlots) sdel[slot * kFSlotStride + lane] = a0 + a1;
        }
    }
    __syncthreads();

    // ---- phase 3: boundary lanes take their corrections; x-sums; owners
    if (kPark && wave < 4) owner_prefetch(g, E0x, E0y, XIN ? xin : nullptr, ob);
    if (wave < 4) {
        const bool interior = valid && I >= 2 && J >= 2 && I <= g.N - 2 && J <= g.N - 2;
        if (!interior) {
            const int rr = (nbr > 0 && J == brow[0]) ? 0 : (nbr > 1 && J == brow[1]) ? 1 : -1;
            const int cc = (nbc > 0 && I == bcol[0]) ? 0 : (nbc > 1 && I == bcol[1]) ? 1 : -1;
            const int slot = (rr >= 0 && cc >= 0) ? 4 * VP + 2 * rr + cc
                             : rr >= 0             ? rr * VP + tx
                                                   : 2 * VP + (cc >= 0 ? cc : 0) * VP + ty;
#pragma unroll
            for (int s = 0; s < kSlots; ++s)
                rv[s] = valid ? sdel[slot * kFSlotStride + s] : T(0);
        }
        T* xs = s_buf;  // 20 values per lane: [(b*2 + c)*2 + parity][lane]
#pragma unroll
        for (int bq = 0; bq < 5; ++bq)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int o = 25 * c + 5 * bq;
                const T ev = rv[o + 4] + row_shl<1>(rv[o + 2]) + row_shl<2>(rv[o + 0]);
                const T od = row_shl<1>(rv[o + 3]) + row_shl<2>(rv[o + 1]);
                const int base = ((bq * 2 + c) * 2) * VNT;
                xs[base + tid] = ev;
                xs[base + VNT + tid] = od;
            }
    }
    __syncthreads();
    if (wave < 4) {
        owner_commit(g, s_buf, E0x, E0y, ob, xout);
        if (valid && tx >= 1 && tx <= VT && ty >= 1 && ty <= VT) {
            const int64_t q = 2 * g.nq2 + int64_t(J) * g.s1 + I;
            xout[q] = ob.p + rv[50];
        }
    }
}

// ---------------------------------------------------------------------------
// Vanka update with the interior apply on the 16x16x4 matrix instructions
// (mfma_patch.h).  Same tile, staging, boundary handling and owner sums as
// vanka_sweep_kernel; wave w processes the patch rows 4w..4w+3 of the tile
// in four rounds of 16 patches, lane l serving patch column l % 16 and
// quarter q = l / 16 of the patch slots.  After the inverse butterflies a
// quarter holds complete rows of its component (u_x rows b, 4-b for q < 2;
// u_y rows b, 4-b for q >= 2 with the centre column taken from quarter
// q - 2 by a cross-half shuffle) or the centre row 2 pieces (q >= 2), so
// the x-sums are DPP row shifts as before; each lane then writes six of the
// 21 per-patch row sums (and unused values to a dummy entry) into the LDS
// exchange, which the owners read after one barrier.
// ---------------------------------------------------------------------------

template <typename T>
struct Mfma16;
template <>
struct Mfma16<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 step(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma16<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 step(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

constexpr int kExchangeEntries = 22;  // 20 row sums, pressure, dummy
constexpr int kMfmaLds = kRRegion + kExchangeEntries * VNT;

template <typename T>
__global__ __launch_bounds__(VNT, 2) void vanka_mfma_kernel(Geom g, const T* __restrict__ rb,
                                                            const T* xin, T* xout,
                                                            const T* __restrict__ dbuf,
                                                            const T* __restrict__ mtab, T scale,
                                                            T t) {
    __shared__ T s_buf[kMfmaLds];
    T* const sr0 = s_buf;
    T* const sr1 = sr0 + kRComp;
    T* const srp = sr1 + kRComp;
    T* const xs = s_buf + kRRegion;
    const int tiles = vanka_tiles(g.N);
    const int ntile = tiles * tiles;
    const int per_xcd = (ntile + 7) / 8;
    const int tlin = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tlin >= ntile) return;
    {  // right-hand side blockIdx.y of a batch
        const int64_t bo = int64_t(blockIdx.y) * g.n;
        rb += bo;
        if (xin) xin += bo;
        xout += bo;
        dbuf += int64_t(blockIdx.y) * n_boundary_patches(g.N) * 64;
    }
    const int E0x = (tlin % tiles) * VT, E0y = (tlin / tiles) * VT;

    // operands of the universal interior operator (one per lane and step)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T a_op[4][4];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk)
#pragma unroll
        for (int c = 0; c < 4; ++c) a_op[blk][c] = mtab[(blk * 4 + c) * 64 + lane];

    stage_residual_region(g, rb, E0x, E0y, scale, t, sr0, sr1, srp);

    // per-lane LDS offsets of the quarter's 15 slots for the first round
    // (patch row 4w); later rounds add two node rows (velocity) or VP (pressure)
    const int j = lane & 15, q = lane >> 4;
    int off[kQuarterValues], slot[kQuarterValues];
#pragma unroll
    for (int k = 0; k < kQuarterValues; ++k) {
        slot[k] = quarter_slot(q, k);
        if (k == 12) {
            off[k] = 2 * kRComp + (4 * w) * VP + j;  // the pressure slot
        } else {
            const int f = slot[k] / 25, rem = slot[k] % 25;
            off[k] = f * kRComp + rr_at(2 * (4 * w) + rem / 5, 2 * j + rem % 5);
        }
    }
    // exchange entries written by this quarter: rows b and 4-b of its
    // component (even, odd), then two row-2 pieces, pressure or dummy
    const int fq = q >> 1, bq = q & 1;
    int ent[6];
    ent[0] = (bq * 2 + fq) * 2;
    ent[1] = ent[0] + 1;
    ent[2] = ((4 - bq) * 2 + fq) * 2;
    ent[3] = ent[2] + 1;
    ent[4] = q == 0 ? 20 : q == 1 ? 21 : (2 * 2 + 0) * 2 + (q - 2);
    ent[5] = q < 2 ? 21 : (2 * 2 + 1) * 2 + (q - 2);
    __syncthreads();

    typedef typename Mfma16<T>::v4 v4;
#pragma unroll
    for (int rho = 0; rho < 4; ++rho) {
        const int ty = 4 * w + rho;
        T in[kQuarterValues];
#pragma unroll
        for (int k = 0; k < kQuarterValues; ++k)
            in[k] = s_buf[off[k] + rho * (k == 12 ? VP : 2 * VRS)];
        T B[4][4];
        quarter_forward(q, in, B);
        T D[4][4];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            v4 acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int c = 0; c < 4; ++c) acc = Mfma16<T>::step(a_op[blk][c], B[blk][c], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) D[blk][v] = acc[v];
        }
        T out[kQuarterValues];
        quarter_inverse(q, D, t, out);

        const int I = E0x - 1 + j, J = E0y - 1 + ty;
        const bool valid = I >= 0 && J >= 0 && I <= g.N && J <= g.N;
        const bool interior = valid && I >= 2 && J >= 2 && I <= g.N - 2 && J <= g.N - 2;
        if (!interior) {
            // boundary patch: corrections precomputed; outside the domain:
            // none (patch 0's values, which exist, times zero)
            const int bi = valid ? boundary_index(I, J, g.N) : 0;
            const T m = valid ? T(1) : T(0);
            const T* __restrict__ src = dbuf + int64_t(bi) * 64;
#pragma unroll
            for (int k = 0; k < kQuarterValues; ++k) out[k] = m * src[slot[k]];
        }
        // centre column of rows b, 4-b: own u_x values (q < 2) or the u_y
        // values of quarter q - 2; centre node of row 2 from quarter 0
        const T o10 = __shfl_xor(out[10], 32);
        const T o11 = __shfl_xor(out[11], 32);
        const T cx = __shfl_xor(q == 0 ? out[13] : T(0), 32);
        const T cy = __shfl_xor(q == 0 ? out[14] : T(0), 32);
        const T c1 = q < 2 ? out[8] : o10;
        const T c2 = q < 2 ? out[9] : o11;
        T val[6];
        val[0] = out[1] + row_shl<1>(c1) + row_shl<2>(out[0]);
        val[1] = row_shl<1>(out[5]) + row_shl<2>(out[4]);
        val[2] = out[3] + row_shl<1>(c2) + row_shl<2>(out[2]);
        val[3] = row_shl<1>(out[7]) + row_shl<2>(out[6]);
        const T sh9 = row_shl<1>(out[9]), sh11 = row_shl<1>(out[11]);
        const T rx = row_shl<2>(out[8]) + (q == 2 ? out[9] : sh9) + row_shl<1>(cx);
        const T ry = row_shl<2>(out[10]) + (q == 2 ? out[11] : sh11) + row_shl<1>(cy);
        val[4] = q == 0 ? out[12] : rx;
        val[5] = ry;
#pragma unroll
        for (int m = 0; m < 6; ++m) xs[ent[m] * VNT + ty * VP + j] = val[m];
    }
    __syncthreads();

    owner_update_velocity(g, xs, E0x, E0y, xin, xout);
    const int tx = threadIdx.x % VP, ty = threadIdx.x / VP;
    const int I = E0x - 1 + tx, J = E0y - 1 + ty;
    const bool valid = I >= 0 && J >= 0 && I <= g.N && J <= g.N;
    if (valid && tx >= 1 && tx <= VT && ty >= 1 && ty <= VT) {
        const int64_t qn = 2 * g.nq2 + int64_t(J) * g.s1 + I;
        xout[qn] = (xin ? xin[qn] : T(0)) + xs[20 * VNT + threadIdx.x];
    }
}

// ---------------------------------------------------------------------------
// Transfers
// ---------------------------------------------------------------------------

// Transfer kernels issue every load before the first use: taps are padded
// to a fixed count with zero weights, and taps that fall on Dirichlet or
// outside nodes read node 0 and get weight zero.

// 1D restriction taps of coarse Q2 node ic: fine offsets and weights (the
// transpose of the Q2 interpolation), padded to five.
__device__ __forceinline__ void q2_restrict_taps(int ic, int (&off)[5], double (&w)[5]) {
    if ((ic & 1) == 0) {
        off[0] = -3; w[0] = -0.125;
        off[1] = -1; w[1] = 0.375;
        off[2] = 0;  w[2] = 1.0;
        off[3] = 1;  w[3] = 0.375;
        off[4] = 3;  w[4] = -0.125;
    } else {
        off[0] = -1; w[0] = 0.75;
        off[1] = 0;  w[1] = 1.0;
        off[2] = 1;  w[2] = 0.75;
        off[3] = 0;  w[3] = 0.0;
        off[4] = 0;  w[4] = 0.0;
    }
}

// Restriction, one thread per coarse Q2 column ic and coarse element row
// jg: the coarse rows 2jg (vertex row) and 2jg+1 (midpoint row), which
// need the fine rows 4jg + {-3, -1, 0, 1, 2, 3}; each fine row is first
// restricted along x (five padded taps), then the rows are combined with
// the 1D weights along y.  The last element row also writes the top
// coarse boundary row (zero).  Pressure: coarse row jg (and Nc on the last
// row) from the 3x3 fine neighbourhood with weights (1/2, 1, 1/2)^2.
template <typename T>
__global__ __launch_bounds__(256) void restrict_kernel(Geom gf, Geom gc, const T* __restrict__ rf,
                                                       T* __restrict__ bc) {
    const int ic = blockIdx.x * 64 + (threadIdx.x & 63);  // 64 x 4 threads per block:
    const int jg = blockIdx.y * 4 + (threadIdx.x >> 6);   // a wave reads whole rows
    if (ic >= gc.s2 || jg >= gc.N) return;
    rf += int64_t(blockIdx.z) * gf.n;  // right-hand side blockIdx.z of a batch
    bc += int64_t(blockIdx.z) * gc.n;
    const bool last = jg == gc.N - 1;
    {
        constexpr int kRow[6] = {-3, -1, 0, 1, 2, 3};
        int ox[5];
        double wx[5];
        q2_restrict_taps(ic, ox, wx);
        const bool col_in = ic > 0 && ic < gc.s2 - 1;
        T vx[6][5], vy[6][5];
        bool ok[6][5];
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                const int i_f = 2 * ic + ox[a], jf = 4 * jg + kRow[r];
                ok[r][a] = col_in && i_f > 0 && jf > 0 && i_f < gf.s2 - 1 && jf < gf.s2 - 1;
                const int64_t qf = ok[r][a] ? int64_t(jf) * gf.s2 + i_f : 0;
                vx[r][a] = rf[qf];
                vy[r][a] = rf[gf.nq2 + qf];
            }
        T tx[6], ty[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            tx[r] = 0;
            ty[r] = 0;
#pragma unroll
            for (int a = 0; a < 5; ++a) {
                const T wa = ok[r][a] ? T(wx[a]) : T(0);
                tx[r] += wa * vx[r][a];
                ty[r] += wa * vy[r][a];
            }
        }
        // vertex row 2jg: fine rows -3, -1, 0, 1, 3 with -1/8, 3/8, 1, 3/8, -1/8
        // midpoint row 2jg+1: fine rows 1, 2, 3 with 3/4, 1, 3/4
        const bool vrow_in = jg > 0;
        const T sxv = T(-0.125) * tx[0] + T(0.375) * tx[1] + tx[2] + T(0.375) * tx[3] +
                      T(-0.125) * tx[5];
        const T syv = T(-0.125) * ty[0] + T(0.375) * ty[1] + ty[2] + T(0.375) * ty[3] +
                      T(-0.125) * ty[5];
        const T sxm = T(0.75) * tx[3] + tx[4] + T(0.75) * tx[5];
        const T sym = T(0.75) * ty[3] + ty[4] + T(0.75) * ty[5];
        const int64_t q0 = int64_t(2 * jg) * gc.s2 + ic;
        bc[q0] = vrow_in ? sxv : T(0);
        bc[gc.nq2 + q0] = vrow_in ? syv : T(0);
        bc[q0 + gc.s2] = sxm;
        bc[gc.nq2 + q0 + gc.s2] = sym;
        if (last) {
            bc[q0 + 2 * gc.s2] = T(0);
            bc[gc.nq2 + q0 + 2 * gc.s2] = T(0);
        }
    }
    if (ic < gc.s1) {
        const T* pf = rf + 2 * gf.nq2;
        T* pc = bc + 2 * gc.nq2;
        for (int jc = jg; jc <= (last ? jg + 1 : jg); ++jc) {
            T v[3][3];
            bool ok[3][3];
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int i_f = 2 * ic + a - 1, jf = 2 * jc + b - 1;
                    ok[b][a] = i_f >= 0 && jf >= 0 && i_f < gf.s1 && jf < gf.s1;
                    v[b][a] = pf[ok[b][a] ? int64_t(jf) * gf.s1 + i_f : 0];
                }
            T sp = 0;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T wyb = b == 1 ? T(1) : T(0.5);
                T t = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const T wxa = a == 1 ? T(1) : T(0.5);
                    t += ok[b][a] ? wxa * v[b][a] : T(0);
                }
                sp += wyb * t;
            }
            pc[int64_t(jc) * gc.s1 + ic] = sp;
        }
    }
}

// Prolongation (x_f += P e_c), one thread per fine Q2 column i and coarse
// element row jg: the fine rows 4jg..4jg+3 interpolate the coarse rows
// 2jg..2jg+2 (each first interpolated along x at column i) with the 1D
// weights of offsets 0..3 in the coarse element.  The top fine row is
// Dirichlet and no thread writes it.  Pressure: fine rows 2jg, 2jg+1 (and
// 2Nc on the last row) at column i, bilinear from the coarse rows jg,
// jg+1.
template <typename T>
__global__ __launch_bounds__(256) void prolong_kernel(Geom gf, Geom gc, const T* __restrict__ ec,
                                                      T* __restrict__ xf) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);  // 64 x 4 threads per block:
    const int jg = blockIdx.y * 4 + (threadIdx.x >> 6);  // a wave reads whole rows
    if (i >= gf.s2 || jg >= gc.N) return;
    ec += int64_t(blockIdx.z) * gc.n;  // right-hand side blockIdx.z of a batch
    xf += int64_t(blockIdx.z) * gf.n;
    {
        int cx[3];
        double wx[3];
        q2_prolong_taps(i, cx, wx);
        const bool col_free = i > 0 && i < gf.s2 - 1;
        T vx[3][3], vy[3][3];
        bool ok[3][3];
        T f0[4], f1[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int64_t q = int64_t(4 * jg + p) * gf.s2 + i;
            f0[p] = xf[q];
            f1[p] = xf[gf.nq2 + q];
        }
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ok[b][a] = !q2_boundary(cx[a], 2 * jg + b, gc.s2);
                const int64_t qc = ok[b][a] ? int64_t(2 * jg + b) * gc.s2 + cx[a] : 0;
                vx[b][a] = ec[qc];
                vy[b][a] = ec[gc.nq2 + qc];
            }
        T tx[3], ty[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            tx[b] = 0;
            ty[b] = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const T wa = ok[b][a] ? T(wx[a]) : T(0);
                tx[b] += wa * vx[b][a];
                ty[b] += wa * vy[b][a];
            }
        }
        // offsets 0..3 of the coarse element: 1D quadratic interpolation
        const T sx[4] = {tx[0], T(0.375) * tx[0] + T(0.75) * tx[1] + T(-0.125) * tx[2], tx[1],
                         T(-0.125) * tx[0] + T(0.75) * tx[1] + T(0.375) * tx[2]};
        const T sy[4] = {ty[0], T(0.375) * ty[0] + T(0.75) * ty[1] + T(-0.125) * ty[2], ty[1],
                         T(-0.125) * ty[0] + T(0.75) * ty[1] + T(0.375) * ty[2]};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            if (!col_free || (jg == 0 && p == 0)) continue;
            const int64_t q = int64_t(4 * jg + p) * gf.s2 + i;
            xf[q] = f0[p] + sx[p];
            xf[gf.nq2 + q] = f1[p] + sy[p];
        }
    }
    if (i < gf.s1) {
        const T* pc = ec + 2 * gc.nq2;
        T* pf = xf + 2 * gf.nq2;
        const int i0 = i / 2, i1 = (i + 1) / 2;
        const bool last = jg == gc.N - 1;
        const int nrow = last ? 3 : 2;
        T fp[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            fp[r] = pf[int64_t(r < nrow ? 2 * jg + r : 2 * jg) * gf.s1 + i];
        const T p00 = pc[int64_t(jg) * gc.s1 + i0], p01 = pc[int64_t(jg) * gc.s1 + i1];
        const T p10 = pc[int64_t(jg + 1) * gc.s1 + i0], p11 = pc[int64_t(jg + 1) * gc.s1 + i1];
        const T r0 = (i & 1) ? T(0.5) * (p00 + p01) : p00;
        const T r1 = (i & 1) ? T(0.5) * (p10 + p11) : p10;
        pf[int64_t(2 * jg) * gf.s1 + i] = fp[0] + r0;
        pf[int64_t(2 * jg + 1) * gf.s1 + i] = fp[1] + T(0.5) * (r0 + r1);
        if (last) pf[int64_t(2 * jg + 2) * gf.s1 + i] = fp[2] + r1;
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

// Transpose of f -> b_F = (M f)_F (the force-dependent part of rhs_kernel):
// grad_f(k) = h^2/900 sum over the free Q2 nodes i within two of k of
// M_ik lambda_u(i), with the interior row stencil of i (every free row is an
// interior row).  One thread per Q2 node, both components; batched over
// blockIdx.y (lambda advances by g.n, grad by 2 nq2).
__global__ __launch_bounds__(256) void rhs_adjoint_kernel(Geom g, const double* __restrict__ lam,
                                                          double* __restrict__ grad) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.z * 4 + (threadIdx.x >> 6);
    if (i >= g.s2 || j >= g.s2) return;
    lam += int64_t(blockIdx.y) * g.n;
    grad += int64_t(blockIdx.y) * 2 * g.nq2;
    double vx[5][5], vy[5][5];
    bool ok[5][5];
#pragma unroll
    for (int b = 0; b < 5; ++b)
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            const int qi = i - (a - 2), qj = j - (b - 2);
            ok[b][a] = qi > 0 && qj > 0 && qi < g.s2 - 1 && qj < g.s2 - 1;
            const int64_t q = ok[b][a] ? int64_t(qj) * g.s2 + qi : 0;
            vx[b][a] = lam[q];
            vy[b][a] = lam[g.nq2 + q];
        }
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int b = 0; b < 5; ++b)
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            // row node (i - ox, j - oy) with offset (ox, oy) = (a - 2, b - 2)
            const int ox = a - 2, oy = b - 2;
            const int c = st_M((j - oy) & 1, oy) * st_M((i - ox) & 1, ox);
            const double w = ok[b][a] ? double(c) : 0.0;
            sx += w * vx[b][a];
            sy += w * vy[b][a];
        }
    const double cm = g.h * g.h / 900.0;
    const int64_t q = int64_t(j) * g.s2 + i;
    grad[q] = cm * sx;
    grad[g.nq2 + q] = cm * sy;
}

// Gradient with respect to a per-element viscosity:
// grad(e) = -sum over both components of lam_e^T L_e x_e on the free Q2
// nodes of element e (L_e the element Laplacian per unit viscosity, 9 x 9).
// One thread per element; batched over blockIdx.y (lam, x by g.n, grad by
// N^2).
__global__ __launch_bounds__(256) void visc_grad_kernel(Geom g, const double* __restrict__ lam,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ grad) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= g.N * g.N) return;
    lam += int64_t(blockIdx.y) * g.n;
    x += int64_t(blockIdx.y) * g.n;
    grad += int64_t(blockIdx.y) * g.N * g.N;
    const int ex = e % g.N, ey = e / g.N;
    double lv[2][9], xv[2][9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int qi = 2 * ex + k % 3, qj = 2 * ey + k / 3;
        const bool free = qi > 0 && qj > 0 && qi < g.s2 - 1 && qj < g.s2 - 1;
        const int64_t q = int64_t(qj) * g.s2 + qi;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            lv[c][k] = free ? lam[c * g.nq2 + q] : 0.0;
            xv[c][k] = free ? x[c * g.nq2 + q] : 0.0;
        }
    }
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int m = 0; m < 9; ++m) {
            const int a = k % 3, b = k / 3, c = m % 3, d = m / 3;
            const int co = kEM[b][d] * kEK[a][c] + kEK[b][d] * kEM[a][c];
            if (co == 0) continue;
            sum += double(co) * (lv[0][k] * xv[0][m] + lv[1][k] * xv[1][m]);
        }
    grad[e] = -sum / 90.0;
}

// Sum of the pressure block of every batch entry: partial sums per block
// (part[entry * G + blk], G = gridDim.x).
__global__ __launch_bounds__(256) void pressure_sum_kernel(Geom g, const double* __restrict__ x,
                                                           double* __restrict__ part) {
    const double* p = x + int64_t(blockIdx.y) * g.n + 2 * g.nq2;
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < g.nq1;
         i += int64_t(gridDim.x) * 256)
        s += p[i];
    __shared__ double red[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        part[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// x_p -= sum / nq1 with the sum of entry blockIdx.y at sums[entry * so]
__global__ __launch_bounds__(256) void pressure_shift_kernel(Geom g, double* __restrict__ x,
                                                             const double* __restrict__ sums,
                                                             int64_t so) {
    double* p = x + int64_t(blockIdx.y) * g.n + 2 * g.nq2;
    const double m = sums[int64_t(blockIdx.y) * so] / double(g.nq1);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < g.nq1;
         i += int64_t(gridDim.x) * 256)
        p[i] -= m;
}

template <typename T>
__global__ __launch_bounds__(256) void coarse_gemv_kernel(int64_t n, const double* __restrict__ C,
                                                          const T* __restrict__ r,
                                                          T* __restrict__ e) {
    const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    r += int64_t(blockIdx.y) * n;  // right-hand side blockIdx.y of a batch
    e += int64_t(blockIdx.y) * n;
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

// Dirichlet lifting: x = b on the Dirichlet DoFs (both velocity components
// at the boundary Q2 nodes), 0 elsewhere, for nb vectors of g.n back to back.
__global__ void lift_kernel(Geom g, const double* __restrict__ b, double* __restrict__ x,
                            int64_t total) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t k = i % g.n;
        bool dir = false;
        if (k < 2 * g.nq2) {
            const int64_t node = k % g.nq2;
            const int qi = int(node % g.s2), qj = int(node / g.s2);
            dir = qi == 0 || qj == 0 || qi == g.s2 - 1 || qj == g.s2 - 1;
        }
        x[i] = dir ? b[i] : 0.0;
    }
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

// out_k = alpha[k * sa] * in_k for the batch vectors k = blockIdx.y
// (in_k at in + k * sin, out_k at out + k * sout); alpha 0 writes zeros
__global__ void scale_batched_kernel(const double* __restrict__ in, int64_t sin,
                                     const double* __restrict__ alpha, int64_t sa,
                                     double* __restrict__ out, int64_t sout, int64_t n) {
    const int64_t k = blockIdx.y;
    const double a = alpha[k * sa];
    in += k * sin;
    out += k * sout;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = a == 0.0 ? 0.0 : a * in[i];  // alpha 0: zeros even where in is not finite
}

// ---------------------------------------------------------------------------
// Krylov: multi-dot, reduction, update, multi-axpy
// ---------------------------------------------------------------------------

// Batched over blockIdx.y: V and w advance by sb, part by k * gridDim.x.
template <int KMAX>
__global__ __launch_bounds__(256) void mdot_partial_kernel(const double* __restrict__ V,
                                                           int64_t ldv, int k,
                                                           const double* __restrict__ w,
                                                           int64_t n,
                                                           double* __restrict__ part, int64_t sb) {
    V += int64_t(blockIdx.y) * sb;
    w += int64_t(blockIdx.y) * sb;
    part += int64_t(blockIdx.y) * k * gridDim.x;
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

// out[v] = sum of the nblk partials of row v; batched over blockIdx.y
// (partials of gridDim.x rows per batch entry, outputs so apart)
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ part,
                                                              int nblk,
                                                              double* __restrict__ out,
                                                              int64_t so) {
    const int v = blockIdx.x;
    part += int64_t(blockIdx.y) * gridDim.x * nblk;
    out += int64_t(blockIdx.y) * so;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) s += part[int64_t(v) * nblk + i];
    __shared__ double red[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[v] = (red[0] + red[1]) + (red[2] + red[3]);
}

// w <- w - V h; part[v * G + blk] = partial of V_v . w_new (v < k) and
// part[k * G + blk] = partial of ||w_new||^2, G = gridDim.x.
template <int KMAX>
__global__ __launch_bounds__(256) void update_dot_kernel(const double* __restrict__ V,
                                                         int64_t ldv, int k,
                                                         const double* __restrict__ h,
                                                         double* __restrict__ w, int64_t n,
                                                         double* __restrict__ part) {
    double hv[KMAX], acc[KMAX];
#pragma unroll
    for (int v = 0; v < KMAX; ++v) {
        hv[v] = v < k ? h[v] : 0.0;
        acc[v] = 0.0;
    }
    double nrm = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        double vv[KMAX];
#pragma unroll
        for (int v = 0; v < KMAX; ++v) vv[v] = v < k ? V[v * ldv + i] : 0.0;
        double s = w[i];
#pragma unroll
        for (int v = 0; v < KMAX; ++v) s -= hv[v] * vv[v];
        w[i] = s;
        nrm += s * s;
#pragma unroll
        for (int v = 0; v < KMAX; ++v) acc[v] += vv[v] * s;
    }
    __shared__ double red[KMAX + 1][4];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < KMAX; ++v) {
        const double t = wave_sum(acc[v]);
        if (lane == 0) red[v][wv] = t;
    }
    const double tn = wave_sum(nrm);
    if (lane == 0) red[KMAX][wv] = tn;
    __syncthreads();
    if (threadIdx.x <= k) {
        const int v = threadIdx.x < k ? threadIdx.x : KMAX;
        part[int64_t(threadIdx.x) * gridDim.x + blockIdx.x] =
            (red[v][0] + red[v][1]) + (red[v][2] + red[v][3]);
    }
}

// out = (w - V h2) / sqrt(nrm2 - |h2|^2): the second Gram-Schmidt
// correction fused with the normalisation (|w - V h2|^2 = nrm2 - |h2|^2 for
// orthonormal V and h2 = V^T w).  Writes zeros if the norm vanishes.
template <int KMAX>
__global__ __launch_bounds__(256) void normalize_kernel(const double* __restrict__ V, int64_t ldv,
                                                        int k, const double* __restrict__ h2,
                                                        const double* __restrict__ nrm2,
                                                        const double* __restrict__ w,
                                                        double* __restrict__ out, int64_t n) {
    double hv[KMAX];
    double hh = 0.0;
#pragma unroll
    for (int v = 0; v < KMAX; ++v) {
        hv[v] = v < k ? h2[v] : 0.0;
        hh += hv[v] * hv[v];
    }
    const double d = nrm2[0] - hh;
    const double scale = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        double s = w[i];
#pragma unroll
        for (int v = 0; v < KMAX; ++v)
            if (v < k) s -= hv[v] * V[v * ldv + i];
        out[i] = s * scale;
    }
}

// ---------------------------------------------------------------------------
// Givens rotations and the stopping test of FGMRES on the device (delayed
// CGS2 Arnoldi steps): one thread per system of a batch, each owning an area
// of `stride` doubles (GivensLayout, kernels.h) that holds the reduced dots
// of pass 1 of the step, the pass-2 coefficients (alpha, gamma, d, sigma),
// two unrotated Hessenberg columns, the rotated columns R (packed), the
// rotations and the rotated right-hand sides.  Step j finalises column j-1
// (H(i,j-1) += s_i / sigma_{j-1}, H(j,j-1) = alpha_j / sigma_{j-1}), redoes its
// rotation and applies it to gbase, then forms column j (provisional,
// H(j+1,j) = sqrt(d)), rotates it and applies its rotation to a copy gv of
// gbase; |gv[j+1]| is the residual estimate.  A system stops at the target,
// on breakdown (d <= 0), at its iteration limit or on a non-finite value.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int packed_col(int j) { return j * (j + 3) / 2; }

// One Givens step of one system (area `a`, GivensLayout), after the
// Gram-Schmidt passes of Arnoldi step j; its summary goes to stat[0..5]
// (estimate, active flag, iterations, kdone, status, |g_kdone|).
__device__ __forceinline__ void givens_step(double* __restrict__ a, int j,
                                            double* __restrict__ stat) {
    using GL = GivensLayout;
    double* sc = a + GL::kScalars;
    if (sc[GL::kActive] == 0.0) return;
    const double* c = a + GL::kDots;
    const double alpha = a[GL::kCoef + 0], gamma = a[GL::kCoef + 1];
    const double d = a[GL::kCoef + 2], sigma = a[GL::kCoef + 3];
    double* cs = a + GL::kCs;
    double* sn = a + GL::kSn;
    double* gb = a + GL::kGbase;
    double* gv = a + GL::kGv;
    double* Hc = a + GL::kHcols + GL::kHcol * (j & 1);
    double* Hp = a + GL::kHcols + GL::kHcol * ((j + 1) & 1);
    auto rotate_column = [&](const double* H, int col) {
        double* R = a + GL::kR + packed_col(col);
        for (int i = 0; i <= col + 1; ++i) R[i] = H[i];
        for (int i = 0; i < col; ++i) {
            const double t = cs[i] * R[i] + sn[i] * R[i + 1];
            R[i + 1] = -sn[i] * R[i] + cs[i] * R[i + 1];
            R[i] = t;
        }
        const double denom = hypot(R[col], R[col + 1]);
        cs[col] = R[col] / denom;
        sn[col] = R[col + 1] / denom;
        R[col] = denom;
        R[col + 1] = 0.0;
    };
    if (j == 0) {
        gb[0] = sc[GL::kBeta];
        for (int i = 1; i < GL::kMaxRestart + 1; ++i) gb[i] = 0.0;
    }
    bool finite = true;
    const double sigma_prev = sc[GL::kSigmaPrev];
    if (j > 0) {  // finalise column j-1
        for (int i = 0; i < j; ++i) Hp[i] += c[j + i] / sigma_prev;
        Hp[j] = alpha / sigma_prev;
        for (int i = 0; i <= j; ++i) finite = finite && isfinite(Hp[i]);
    }
    for (int i = 0; i < j; ++i) Hc[i] = c[i];
    Hc[j] = gamma;
    const double hnext = d > 0.0 ? sqrt(d) : 0.0;
    sc[GL::kSigmaPrev] = sigma;
    for (int i = 0; i <= j; ++i) finite = finite && isfinite(Hc[i]);
    Hc[j + 1] = hnext;
    sc[GL::kIters] += 1.0;
    if (!finite || !isfinite(hnext)) {
        sc[GL::kActive] = 0.0;
        sc[GL::kStatus] = 1.0;  // non-finite
        sc[GL::kEst] = __builtin_nan("");
    } else {
        if (j > 0) {
            rotate_column(Hp, j - 1);
            gb[j] = -sn[j - 1] * gb[j - 1];
            gb[j - 1] = cs[j - 1] * gb[j - 1];
        }
        rotate_column(Hc, j);
        for (int i = 0; i <= j + 1; ++i) gv[i] = gb[i];
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
        sc[GL::kKdone] = double(j + 1);
        const double res = fabs(gv[j + 1]);
        sc[GL::kEst] = res / sc[GL::kBeta0];
        if (res <= sc[GL::kTarget] || hnext == 0.0 || sc[GL::kIters] >= sc[GL::kMaxIters])
            sc[GL::kActive] = 0.0;
    }
    stat[0] = sc[GL::kEst];
    stat[1] = sc[GL::kActive];
    stat[2] = sc[GL::kIters];
    stat[3] = sc[GL::kKdone];
    stat[4] = sc[GL::kStatus];
    stat[5] = fabs(gv[int(sc[GL::kKdone])]);
}

// Start of a restart cycle: the per-system values the host staged in
// init[8k..8k+7] (beta0, target, beta, estimate, active, iterations,
// iteration limit, 1/beta) into each area, with the Givens state reset.
__global__ __launch_bounds__(64) void givens_init_kernel(double* __restrict__ area, int64_t stride,
                                                         const double* __restrict__ init,
                                                         double* __restrict__ stat, int nsys) {
    using GL = GivensLayout;
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k >= nsys) return;
    double* a = area + int64_t(k) * stride;
    double* sc = a + GL::kScalars;
    const double* in = init + 8 * k;
    sc[GL::kBeta0] = in[0];
    sc[GL::kTarget] = in[1];
    sc[GL::kBeta] = in[2];
    sc[GL::kEst] = in[3];
    sc[GL::kActive] = in[4];
    sc[GL::kIters] = in[5];
    sc[GL::kMaxIters] = in[6];
    a[GL::kScale] = in[7];
    sc[GL::kSigmaPrev] = 0.0;
    sc[GL::kKdone] = 0.0;
    sc[GL::kStatus] = 0.0;
    sc[GL::kCycled] = in[4];
    a[GL::kGv] = 0.0;
    double* st = stat + 8 * k;
    st[0] = in[3];
    st[1] = in[4];
    st[2] = in[5];
    st[3] = 0.0;
    st[4] = 0.0;
    st[5] = 0.0;
    st[6] = in[4];
}

// y = R^{-1} gv for the k = kdone columns of each system that ran in this
// cycle (cycled != 0), zeros up to kmax (the columns x += Z y reads).  One
// workgroup per system: R and g are staged in LDS, one thread substitutes.
__global__ __launch_bounds__(64) void givens_solve_kernel(double* __restrict__ area,
                                                          int64_t stride, int kmax) {
    using GL = GivensLayout;
    constexpr int kRSize = GL::kMaxRestart * (GL::kMaxRestart + 3) / 2;
    __shared__ double sR[kRSize], sg[GL::kMaxRestart + 1], sy[GL::kMaxRestart];
    double* a = area + int64_t(blockIdx.x) * stride;
    for (int i = threadIdx.x; i < kRSize; i += 64) sR[i] = a[GL::kR + i];
    if (threadIdx.x < GL::kMaxRestart + 1) sg[threadIdx.x] = a[GL::kGv + threadIdx.x];
    const double* sc = a + GL::kScalars;
    const int kk = sc[GL::kCycled] != 0.0 ? int(sc[GL::kKdone]) : 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = kk - 1; i >= 0; --i) {
            double acc = sg[i];
            for (int l = i + 1; l < kk; ++l) acc -= sR[packed_col(l) + i] * sy[l];
            sy[i] = acc / sR[packed_col(i) + i];
        }
    }
    __syncthreads();
    if (threadIdx.x < kmax) a[GL::kY + threadIdx.x] = threadIdx.x < kk ? sy[threadIdx.x] : 0.0;
}

// Delayed classical Gram-Schmidt with reorthogonalisation (the DCGS2 of
// Bielich, Langou, Thomas, Swirydowicz, Yamazaki and Boman): the second
// pass for basis vector j shares its sweep with the first pass for
// w = A z_j.  V holds the j final vectors, u the once-orthogonalised,
// unnormalised vector j.  Pass 1 leaves partials (G = gridDim.x) of
//   rows [0, j)   V^T w  (h)        rows [j, 2j)  V^T u  (s)
//   row 2j  u.u,  row 2j+1  u.w,  row 2j+2  w.w
// in part[row * G + blk].
template <int KMAX>
__global__ __launch_bounds__(256) void dcgs_dots_kernel(const double* __restrict__ V, int64_t ldv,
                                                        int j, const double* __restrict__ u,
                                                        const double* __restrict__ w, int64_t n,
                                                        double* __restrict__ part, int64_t sb) {
    {  // batch entry blockIdx.y: vectors sb apart, 2j+3 rows of partials each
        const int64_t bo = int64_t(blockIdx.y) * sb;
        V += bo;
        u += bo;
        w += bo;
        part += int64_t(blockIdx.y) * (2 * j + 3) * gridDim.x;
    }
    double aw[KMAX], au[KMAX];
    double uu = 0.0, uw = 0.0, ww = 0.0;
#pragma unroll
    for (int v = 0; v < KMAX; ++v) aw[v] = au[v] = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        double vv[KMAX];
#pragma unroll
        for (int v = 0; v < KMAX; ++v) vv[v] = v < j ? V[v * ldv + i] : 0.0;
        const double ui = u[i], wi = w[i];
        uu += ui * ui;
        uw += ui * wi;
        ww += wi * wi;
#pragma unroll
        for (int v = 0; v < KMAX; ++v) {
            aw[v] += vv[v] * wi;
            au[v] += vv[v] * ui;
        }
    }
    __shared__ double red[2 * KMAX + 3][4];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < KMAX; ++v) {
        if (v >= j) break;
        const double a = wave_sum(aw[v]), b = wave_sum(au[v]);
        if (lane == 0) {
            red[v][wv] = a;
            red[KMAX + v][wv] = b;
        }
    }
    {
        const double a = wave_sum(uu), b = wave_sum(uw), c = wave_sum(ww);
        if (lane == 0) {
            red[2 * KMAX][wv] = a;
            red[2 * KMAX + 1][wv] = b;
            red[2 * KMAX + 2][wv] = c;
        }
    }
    __syncthreads();
    const int row = threadIdx.x;
    if (row < 2 * j + 3) {
        const int r = row < j ? row : row < 2 * j ? KMAX + row - j : 2 * KMAX + row - 2 * j;
        part[int64_t(row) * gridDim.x + blockIdx.x] = (red[r][0] + red[r][1]) + (red[r][2] + red[r][3]);
    }
}

// Pass 2 of the delayed scheme from the reduced values c of pass 1:
//   alpha = sqrt(u.u - |s|^2),  v_j = (u - V s) / alpha   (written over u)
//   gamma = v_j . w = (u.w - s.h) / alpha
//   d = |w - V h - gamma v_j|^2 = w.w - |h|^2 - gamma^2
//   next = (w - V h - gamma v_j) / sqrt(d)   (zeros if d <= 0)
// Every block derives the same coefficients; block 0 stores
// (alpha, gamma, d, 1/sqrt(d)) in cf for the Hessenberg matrix.
template <int KMAX>
__global__ __launch_bounds__(256) void dcgs_update_kernel(const double* __restrict__ V, int64_t ldv,
                                                          int j, const double* __restrict__ c,
                                                          double* uv, const double* __restrict__ w,
                                                          double* __restrict__ next, int64_t n,
                                                          double* __restrict__ cf, int64_t sb,
                                                          int64_t sc, float* __restrict__ next32,
                                                          double* __restrict__ garea,
                                                          double* __restrict__ gstat) {
    {  // batch entry blockIdx.y: vectors sb apart, coefficients sc apart
        const int64_t bo = int64_t(blockIdx.y) * sb;
        V += bo;
        uv += bo;
        w += bo;
        next += bo;
        if (next32) next32 += bo;
        c += int64_t(blockIdx.y) * sc;
        cf += int64_t(blockIdx.y) * sc;
    }
    double hv[KMAX], sv[KMAX];
    double ss = 0.0, hh = 0.0, sh = 0.0;
#pragma unroll
    for (int v = 0; v < KMAX; ++v) {
        hv[v] = v < j ? c[v] : 0.0;
        sv[v] = v < j ? c[j + v] : 0.0;
        ss += sv[v] * sv[v];
        hh += hv[v] * hv[v];
        sh += sv[v] * hv[v];
    }
    const double uu = c[2 * j], uw = c[2 * j + 1], ww = c[2 * j + 2];
    const double a2 = uu - ss;
    const double alpha = a2 > 0.0 ? sqrt(a2) : 0.0;
    const double ra = alpha > 0.0 ? 1.0 / alpha : 0.0;
    const double gamma = (uw - sh) * ra;
    const double d = ww - hh - gamma * gamma;
    const double sigma = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cf[0] = alpha;
        cf[1] = gamma;
        cf[2] = d;
        cf[3] = sigma;
    }
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        double vv[KMAX];
#pragma unroll
        for (int v = 0; v < KMAX; ++v) vv[v] = v < j ? V[v * ldv + i] : 0.0;
        const double ui = uv[i], wi = w[i];
        double ps = 0.0, ph = 0.0;
#pragma unroll
        for (int v = 0; v < KMAX; ++v) {
            ps += sv[v] * vv[v];
            ph += hv[v] * vv[v];
        }
        const double vj = (ui - ps) * ra;
        uv[i] = vj;
        const double nx = ((wi - ph) - gamma * vj) * sigma;
        next[i] = nx;
        if (next32) next32[i] = float(nx);
    }
    // block 0 of each batch entry: the entry's Givens step, on a copy of its
    // area in LDS (one thread; global round trips would serialise it)
    if (garea && blockIdx.x == 0) {
        using GL = GivensLayout;
        __shared__ double gl[GL::kSize];
        double* a = garea + int64_t(blockIdx.y) * sc;
        constexpr int kState = GL::kScalars + GL::kNumScalars - GL::kCs;
        for (int i = threadIdx.x; i < 2 * j + 3; i += 256) gl[GL::kDots + i] = a[GL::kDots + i];
        for (int i = threadIdx.x; i < kState; i += 256) gl[GL::kCs + i] = a[GL::kCs + i];
        if (threadIdx.x == 0) {
            gl[GL::kCoef + 0] = alpha;
            gl[GL::kCoef + 1] = gamma;
            gl[GL::kCoef + 2] = d;
            gl[GL::kCoef + 3] = sigma;
        }
        __syncthreads();
        if (threadIdx.x == 0) givens_step(gl, j, gstat + 8 * blockIdx.y);
        __syncthreads();
        for (int i = threadIdx.x; i < kState; i += 256) a[GL::kCs + i] = gl[GL::kCs + i];
    }
}

// w <- w - V h (no reduction)
template <int KMAX>
__global__ __launch_bounds__(256) void update_kernel(const double* __restrict__ V, int64_t ldv,
                                                     int k, const double* __restrict__ h,
                                                     double* __restrict__ w, int64_t n) {
    double hv[KMAX];
#pragma unroll
    for (int v = 0; v < KMAX; ++v) hv[v] = v < k ? h[v] : 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        double s = w[i];
#pragma unroll
        for (int v = 0; v < KMAX; ++v)
            if (v < k) s -= hv[v] * V[v * ldv + i];
        w[i] = s;
    }
}

template <int KMAX>
__global__ __launch_bounds__(256) void axpy_multi_kernel(const double* __restrict__ Z, int64_t ldz,
                                                         int k, const double* __restrict__ y,
                                                         double* __restrict__ x, int64_t n,
                                                         int64_t sb, int64_t sy) {
    Z += int64_t(blockIdx.y) * sb;  // batch entry blockIdx.y
    x += int64_t(blockIdx.y) * sb;
    y += int64_t(blockIdx.y) * sy;
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

// Boundary patches per wavefront: `per` (1, 2, 4 or 8) if given, else about
// one wavefront per SIMD (1024) on the large levels, where the coefficient
// rows dominate the traffic.
int boundary_patches_per_wave(int nb, int per) {
    if (per == 1 || per == 2 || per == 4 || per == 8) return per;
    const int q = nb / 1024;
    return q >= 8 ? 8 : q >= 4 ? 4 : q >= 2 ? 2 : 1;
}

int elementwise_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return int(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
//
// The build compiles this file twice, with VKMG_KERNEL_UNIT = 64 (the FP64
// launchers and everything not tied to a precision; machine scheduling that
// keeps memory clauses together, under which the residual kernel does not
// spill) and with VKMG_KERNEL_UNIT = 32 (the FP32 launchers; the compiler's
// default scheduling, faster for them).  Without the macro one unit holds
// everything.
// ---------------------------------------------------------------------------

#if !defined(VKMG_KERNEL_UNIT) || VKMG_KERNEL_UNIT == 64
#define VKMG_UNIT64 1
#else
#define VKMG_UNIT64 0
#endif
#if !defined(VKMG_KERNEL_UNIT) || VKMG_KERNEL_UNIT == 32
#define VKMG_UNIT32 1
#else
#define VKMG_UNIT32 0
#endif

template <typename Tx, typename T>
void launch_residual(const Geom& g, const T* b, const Tx* x, T* r, int mode, hipStream_t s,
                     int nb, const T* nue) {
    const int tiles = (g.N + 1 + RT - 1) / RT;
    const dim3 grid(8 * ((tiles * tiles + 7) / 8), nb);
    if (nue) {
        if (mode == 0)
            residual_kernel<0, Tx, T, true><<<grid, RNT, 0, s>>>(g, b, x, r, nue);
        else
            residual_kernel<1, Tx, T, true><<<grid, RNT, 0, s>>>(g, b, x, r, nue);
    } else if (mode == 0) {
        residual_kernel<0, Tx, T><<<grid, RNT, 0, s>>>(g, b, x, r);
    } else {
        residual_kernel<1, Tx, T><<<grid, RNT, 0, s>>>(g, b, x, r);
    }
}
#if VKMG_UNIT64
template void launch_residual<double, double>(const Geom&, const double*, const double*, double*,
                                              int, hipStream_t, int, const double*);
#endif

#if VKMG_UNIT32
void launch_apply_widen(const Geom& g, const float* x, double* y, double* x64, hipStream_t s,
                        const double* nue, int nb) {
    const int tiles = (g.N + 1 + RT - 1) / RT;
    const dim3 grid(8 * ((tiles * tiles + 7) / 8), nb);
    if (nue)
        residual_kernel<1, float, double, true, false, true><<<grid, RNT, 0, s>>>(
            g, nullptr, x, y, nue, Geom{}, nullptr, x64);
    else
        residual_kernel<1, float, double, false, false, true><<<grid, RNT, 0, s>>>(
            g, nullptr, x, y, nullptr, Geom{}, nullptr, x64);
}
#endif

template <typename T>
void launch_residual_prolong(const Geom& g, const Geom& gc, const T* b, const T* x, const T* ec,
                             T* x2, T* r, hipStream_t s, int nb, const T* nue) {
    const int tiles = (g.N + 1 + RT - 1) / RT;
    const dim3 grid(8 * ((tiles * tiles + 7) / 8), nb);
    if (nue)
        residual_kernel<0, T, T, true, true><<<grid, RNT, 0, s>>>(g, b, x, r, nue, gc, ec, x2);
    else
        residual_kernel<0, T, T, false, true><<<grid, RNT, 0, s>>>(g, b, x, r, nullptr, gc, ec, x2);
}
#if VKMG_UNIT64
template void launch_residual_prolong<double>(const Geom&, const Geom&, const double*,
                                              const double*, const double*, double*, double*,
                                              hipStream_t, int, const double*);
#endif
#if VKMG_UNIT32
template void launch_residual_prolong<float>(const Geom&, const Geom&, const float*, const float*,
                                             const float*, float*, float*, hipStream_t, int,
                                             const float*);
template void launch_residual<float, float>(const Geom&, const float*, const float*, float*, int,
                                            hipStream_t, int, const float*);
#endif

#if VKMG_UNIT64
void launch_rhs(const Geom& g, const double* f, const double* gd, double* b, hipStream_t s,
                int nb) {
    const dim3 grid((g.N + 1 + 15) / 16, (g.N + 1 + 15) / 16, nb);
    rhs_kernel<<<grid, 256, 0, s>>>(g, f, gd, b);
}
#endif

template <typename T>
void launch_bs_relax(const Geom& g, const T* r, const T* xin, T* xout, T* prhs, T* dp, T* vtmp,
                     double t, double omega, double jacobi_weight, int jacobi_sweeps,
                     hipStream_t s, int nb) {
    const int tiles = (g.N + 1 + BT - 1) / BT;
    const dim3 grid(8 * ((tiles * tiles + 7) / 8), nb);
    const T inv_t = T(1.0 / t), wj = T(jacobi_weight);
    bs_div_kernel<T, 0><<<grid, BNT, 0, s>>>(g, r, prhs, dp, inv_t, wj);
    for (int k = 1; k < jacobi_sweeps; ++k) {
        bs_grad_kernel<T, 0><<<grid, BNT, 0, s>>>(g, dp, nullptr, nullptr, vtmp, T(0), T(0));
        bs_div_kernel<T, 1><<<grid, BNT, 0, s>>>(g, vtmp, prhs, dp, inv_t, wj);
    }
    bs_grad_kernel<T, 1><<<grid, BNT, 0, s>>>(g, dp, r, xin, xout, T(omega / t), T(omega));
}
#if VKMG_UNIT64
template void launch_bs_relax<double>(const Geom&, const double*, const double*, double*, double*,
                                      double*, double*, double, double, double, int, hipStream_t,
                                      int);
#endif
#if VKMG_UNIT32
template void launch_bs_relax<float>(const Geom&, const float*, const float*, float*, float*,
                                     float*, float*, double, double, double, int, hipStream_t,
                                     int);
#endif

#if VKMG_UNIT64
void launch_rhs_adjoint(const Geom& g, const double* lam, double* grad, hipStream_t s, int nb) {
    const dim3 grid((g.s2 + 63) / 64, nb, (g.s2 + 3) / 4);
    rhs_adjoint_kernel<<<grid, 256, 0, s>>>(g, lam, grad);
}

void launch_visc_grad(const Geom& g, const double* lam, const double* x, double* grad,
                      hipStream_t s, int nb) {
    const int ne = g.N * g.N;
    visc_grad_kernel<<<dim3((ne + 255) / 256, nb), 256, 0, s>>>(g, lam, x, grad);
}

void launch_pressure_mean_zero(const Geom& g, double* x, double* part, double* sums, int64_t so,
                               hipStream_t s, int nb) {
    constexpr int kBlocks = 256;
    pressure_sum_kernel<<<dim3(kBlocks, nb), 256, 0, s>>>(g, x, part);
    reduce_partials_kernel<<<dim3(1, nb), 256, 0, s>>>(part, kBlocks, sums, so);
    pressure_shift_kernel<<<dim3(kBlocks, nb), 256, 0, s>>>(g, x, sums, so);
}
#endif

template <typename T>
void launch_vanka_simple(const Geom& g, const T* r, const T* xin, T* xout, const T* tables,
                         T* dbuf, hipStream_t s, int nb) {
    const int np = (g.N + 1) * (g.N + 1);
    vanka_patch_kernel<T><<<dim3((np + 3) / 4, nb), 256, 0, s>>>(g, r, tables, dbuf);
    const int ntile = vanka_tiles(g.N) * vanka_tiles(g.N);
    const dim3 grid(8 * ((ntile + 7) / 8), nb);
    vanka_sweep_kernel<T, true><<<grid, VNT, 0, s>>>(g, r, xin, xout, dbuf, T(0), T(0));
}
#if VKMG_UNIT64
template void launch_vanka_simple<double>(const Geom&, const double*, const double*, double*,
                                          const double*, double*, hipStream_t, int);
#endif
#if VKMG_UNIT32
template void launch_vanka_simple<float>(const Geom&, const float*, const float*, float*,
                                         const float*, float*, hipStream_t, int);
#endif

#if VKMG_UNIT64
int64_t vanka_boundary_scratch(int N) { return int64_t(n_boundary_patches(N)) * 64; }
#endif

template <typename T>
void launch_vanka_boundary(const Geom& g, const T* r, const T* table, T* dbuf, hipStream_t s,
                           int nrhs, int per_wave) {
    const int nb = n_boundary_patches(g.N);
    const int per = boundary_patches_per_wave(nb * nrhs, per_wave);
    const dim3 bgrid((nb + 4 * per - 1) / (4 * per), nrhs);
    if (per == 8)
        vanka_boundary_kernel<T, 8><<<bgrid, 256, 0, s>>>(g, r, table, dbuf);
    else if (per == 4)
        vanka_boundary_kernel<T, 4><<<bgrid, 256, 0, s>>>(g, r, table, dbuf);
    else if (per == 2)
        vanka_boundary_kernel<T, 2><<<bgrid, 256, 0, s>>>(g, r, table, dbuf);
    else
        vanka_boundary_kernel<T, 1><<<bgrid, 256, 0, s>>>(g, r, table, dbuf);
}
#if VKMG_UNIT64
template void launch_vanka_boundary<double>(const Geom&, const double*, const double*, double*,
                                            hipStream_t, int, int);
#endif
#if VKMG_UNIT32
template void launch_vanka_boundary<float>(const Geom&, const float*, const float*, float*,
                                           hipStream_t, int, int);
#endif

template <typename T>
void launch_vanka_tiles(const Geom& g, const T* r, const T* xin, T* xout, const T* mtab,
                        const T* dbuf, double omega, bool mfma, hipStream_t s, int nrhs,
                        bool park) {
    const int ntile = vanka_tiles(g.N) * vanka_tiles(g.N);
    const dim3 grid(8 * ((ntile + 7) / 8), nrhs);
    if (mfma)
        vanka_mfma_kernel<T><<<grid, VNT, 0, s>>>(g, r, xin, xout, dbuf, mtab, T(omega / g.nu),
                                                  T(g.nu / g.h));
    else if (std::is_same<T, double>::value && park)
        vanka_sweep_kernel<T, false, true><<<grid, VNT, 0, s>>>(g, r, xin, xout, dbuf,
                                                                T(omega / g.nu), T(g.nu / g.h));
    else
        vanka_sweep_kernel<T><<<grid, VNT, 0, s>>>(g, r, xin, xout, dbuf, T(omega / g.nu),
                                                   T(g.nu / g.h));
}
#if VKMG_UNIT64
template void launch_vanka_tiles<double>(const Geom&, const double*, const double*, double*,
                                         const double*, const double*, double, bool, hipStream_t,
                                         int, bool);
#endif
#if VKMG_UNIT32
template void launch_vanka_tiles<float>(const Geom&, const float*, const float*, float*,
                                        const float*, const float*, double, bool, hipStream_t,
                                        int, bool);
#endif

template <typename T>
void launch_vanka_fused(const Geom& g, const T* b, const T* xin, T* xout, const T* table,
                        double omega, hipStream_t s, int nrhs) {
    const int ntile = vanka_tiles(g.N) * vanka_tiles(g.N);
    const dim3 grid(8 * ((ntile + 7) / 8), nrhs);
    if (xin)
        vanka_fused_kernel<T, true><<<grid, FNT, 0, s>>>(g, b, xin, xout, table, T(omega / g.nu),
                                                         T(g.nu / g.h));
    else
        vanka_fused_kernel<T, false><<<grid, FNT, 0, s>>>(g, b, xin, xout, table,
                                                          T(omega / g.nu), T(g.nu / g.h));
}
#if VKMG_UNIT64
template void launch_vanka_fused<double>(const Geom&, const double*, const double*, double*,
                                         const double*, double, hipStream_t, int);
#endif
#if VKMG_UNIT32
template void launch_vanka_fused<float>(const Geom&, const float*, const float*, float*,
                                        const float*, double, hipStream_t, int);
#endif
#if VKMG_UNIT64
int vanka_fused_min_n() { return kFusedMinN; }
#endif

template <typename T>
void launch_vanka_update(const Geom& g, const T* r, const T* xin, T* xout, const T* table,
                         const T* mtab, T* dbuf, double omega, bool mfma, hipStream_t s,
                         int nrhs, bool park, int per_wave) {
    launch_vanka_boundary<T>(g, r, table, dbuf, s, nrhs, per_wave);
    launch_vanka_tiles<T>(g, r, xin, xout, mtab, dbuf, omega, mfma, s, nrhs, park);
}
#if VKMG_UNIT64
template void launch_vanka_update<double>(const Geom&, const double*, const double*, double*,
                                          const double*, const double*, double*, double, bool,
                                          hipStream_t, int, bool, int);
#endif
#if VKMG_UNIT32
template void launch_vanka_update<float>(const Geom&, const float*, const float*, float*,
                                         const float*, const float*, float*, double, bool,
                                         hipStream_t, int, bool, int);
#endif

template <typename T>
void launch_restrict(const Geom& gf, const Geom& gc, const T* rf, T* bc, hipStream_t s, int nb) {
    const dim3 grid((gc.s2 + 63) / 64, (gc.N + 3) / 4, nb);
    restrict_kernel<T><<<grid, 256, 0, s>>>(gf, gc, rf, bc);
}
#if VKMG_UNIT64
template void launch_restrict<double>(const Geom&, const Geom&, const double*, double*, hipStream_t,
                                      int);
#endif
#if VKMG_UNIT32
template void launch_restrict<float>(const Geom&, const Geom&, const float*, float*, hipStream_t,
                                     int);
#endif

template <typename T>
void launch_prolong_add(const Geom& gf, const Geom& gc, const T* ec, T* xf, hipStream_t s, int nb) {
    const dim3 grid((gf.s2 + 63) / 64, (gc.N + 3) / 4, nb);
    prolong_kernel<T><<<grid, 256, 0, s>>>(gf, gc, ec, xf);
}
#if VKMG_UNIT64
template void launch_prolong_add<double>(const Geom&, const Geom&, const double*, double*,
                                         hipStream_t, int);
#endif
#if VKMG_UNIT32
template void launch_prolong_add<float>(const Geom&, const Geom&, const float*, float*,
                                        hipStream_t, int);
#endif

template <typename T>
void launch_coarse_gemv(int64_t n, const double* C, const T* r, T* e, hipStream_t s, int nb) {
    const dim3 grid(int((n + 3) / 4), nb);
    coarse_gemv_kernel<T><<<grid, 256, 0, s>>>(n, C, r, e);
}
#if VKMG_UNIT64
template void launch_coarse_gemv<double>(int64_t, const double*, const double*, double*,
                                         hipStream_t, int);
#endif
#if VKMG_UNIT32
template void launch_coarse_gemv<float>(int64_t, const double*, const float*, float*, hipStream_t,
                                        int);
#endif

template <typename T>
void launch_fill_zero(T* x, int64_t n, hipStream_t s) {
    fill_zero_kernel<T><<<elementwise_blocks(n), 256, 0, s>>>(x, n);
}
#if VKMG_UNIT64
template void launch_fill_zero<double>(double*, int64_t, hipStream_t);
#endif
#if VKMG_UNIT32
template void launch_fill_zero<float>(float*, int64_t, hipStream_t);
#endif

template <typename Ti, typename To>
void launch_cast(const Ti* in, To* out, int64_t n, hipStream_t s) {
    cast_kernel<Ti, To><<<elementwise_blocks(n), 256, 0, s>>>(in, out, n);
}
#if VKMG_UNIT32
template void launch_cast<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_cast<float, double>(const float*, double*, int64_t, hipStream_t);
#endif

#if VKMG_UNIT64
void launch_lift(const Geom& g, const double* b, double* x, hipStream_t s, int nb) {
    const int64_t total = g.n * nb;
    lift_kernel<<<elementwise_blocks(total), 256, 0, s>>>(g, b, x, total);
}

void launch_scale(const double* in, double alpha, double* out, int64_t n, hipStream_t s) {
    scale_kernel<<<elementwise_blocks(n), 256, 0, s>>>(in, alpha, out, n);
}
#endif

#define VKMG_KDISPATCH(k, KERNEL, ...)                                     \
    do {                                                                   \
        if ((k) <= 4) KERNEL<4><<<kgrid, 256, 0, s>>>(__VA_ARGS__);        \
        else if ((k) <= 8) KERNEL<8><<<kgrid, 256, 0, s>>>(__VA_ARGS__);   \
        else if ((k) <= 16) KERNEL<16><<<kgrid, 256, 0, s>>>(__VA_ARGS__); \
        else KERNEL<32><<<kgrid, 256, 0, s>>>(__VA_ARGS__);                \
    } while (0)

// The Krylov kernels keep up to 32 coefficients in registers; longer
// bases are processed in chunks of 32 vectors (single right-hand side).
constexpr int kChunk = 32;

#if VKMG_UNIT64
void launch_givens_init(double* area, int64_t stride, const double* init, double* stat, int nsys,
                        hipStream_t s) {
    givens_init_kernel<<<(nsys + 63) / 64, 64, 0, s>>>(area, stride, init, stat, nsys);
}

void launch_givens_solve(double* area, int64_t stride, int kmax, int nsys, hipStream_t s) {
    givens_solve_kernel<<<nsys, 64, 0, s>>>(area, stride, kmax);
}
#endif

// Every batch entry is reduced over the same kDotBlocks partial sums as a
// single right-hand side, so batched dot products (and with them the whole
// batched solve) are bitwise those of single solves.
#if VKMG_UNIT64
int dot_blocks(int) { return kDotBlocks; }

void launch_scale_batched(const double* in, int64_t sin, const double* alpha, int64_t sa,
                          double* out, int64_t sout, int64_t n, int nb, hipStream_t s) {
    int bx = elementwise_blocks(n) / nb;
    const dim3 grid(bx < 1 ? 1 : bx, nb);
    scale_batched_kernel<<<grid, 256, 0, s>>>(in, sin, alpha, sa, out, sout, n);
}

void launch_mdot_partial(const double* V, int64_t ldv, int k, const double* w, int64_t n,
                         double* part, hipStream_t s, int nb, int64_t sb) {
    const dim3 kgrid(dot_blocks(nb), nb);
    for (int c0 = 0; c0 < k; c0 += kChunk) {
        const int kc = k - c0 < kChunk ? k - c0 : kChunk;
        VKMG_KDISPATCH(kc, mdot_partial_kernel, V + c0 * ldv, ldv, kc, w, n,
                       part + int64_t(c0) * kDotBlocks, sb);
    }
}

void launch_reduce_partials(const double* part, int k, double* out, hipStream_t s, int nb,
                            int64_t so) {
    reduce_partials_kernel<<<dim3(k, nb), 256, 0, s>>>(part, dot_blocks(nb), out, so);
}

void launch_update(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t n,
                   hipStream_t s) {
    const dim3 kgrid(kDotBlocks, 1);
    for (int c0 = 0; c0 < k; c0 += kChunk) {
        const int kc = k - c0 < kChunk ? k - c0 : kChunk;
        VKMG_KDISPATCH(kc, update_kernel, V + c0 * ldv, ldv, kc, h + c0, w, n);
    }
}

void launch_update_dot(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t n,
                       double* part, hipStream_t s) {
    const dim3 kgrid(kDotBlocks, 1);
    VKMG_KDISPATCH(k, update_dot_kernel, V, ldv, k, h, w, n, part);
}

void launch_normalize(const double* V, int64_t ldv, int k, const double* h2, const double* nrm2,
                      const double* w, double* out, int64_t n, hipStream_t s) {
    const dim3 kgrid(kDotBlocks, 1);
    VKMG_KDISPATCH(k, normalize_kernel, V, ldv, k, h2, nrm2, w, out, n);
}

void launch_dcgs_dots(const double* V, int64_t ldv, int j, const double* u, const double* w,
                      int64_t n, double* part, hipStream_t s, int nb, int64_t sb) {
    const dim3 kgrid(dot_blocks(nb), nb);
    VKMG_KDISPATCH(j, dcgs_dots_kernel, V, ldv, j, u, w, n, part, sb);
}

void launch_dcgs_update(const double* V, int64_t ldv, int j, const double* c, double* u,
                        const double* w, double* next, int64_t n, double* cf, hipStream_t s,
                        int nb, int64_t sb, int64_t sc, float* next32, double* garea,
                        double* gstat) {
    const dim3 kgrid(dot_blocks(nb), nb);
    VKMG_KDISPATCH(j, dcgs_update_kernel, V, ldv, j, c, u, w, next, n, cf, sb, sc, next32, garea,
                   gstat);
}

void launch_axpy_multi(const double* Z, int64_t ldz, int k, const double* y, double* x, int64_t n,
                       hipStream_t s, int nb, int64_t sb, int64_t sy) {
    const dim3 kgrid(dot_blocks(nb), nb);
    for (int c0 = 0; c0 < k; c0 += kChunk) {
        const int kc = k - c0 < kChunk ? k - c0 : kChunk;
        VKMG_KDISPATCH(kc, axpy_multi_kernel, Z + c0 * ldz, ldz, kc, y + c0, x, n, sb, sy);
    }
}
#endif

}  // namespace vkmg
