// Host-side setup of the vkmg library, FP64.
//
// * Element matrices of the Q2-Q1 Taylor-Hood pair on a square element of
//   side h, from the closed-form 1D factors (paper, section "Discretization":
//   L_ij = a(psi_j, psi_i) with a(u,v) = nu int grad u : grad v, and
//   B_kj = b(psi_j, phi_k) with b(v,q) = -int q div v):
//     1D quadratic stiffness  K1 = (1/3h) [[7,-8,1],[-8,16,-8],[1,-8,7]]
//     1D quadratic mass       M1 = (h/30) [[4,2,-1],[2,16,2],[-1,2,4]]
//     mixed  G[c][a]  = int phi_c psi_a'  = (1/6) [[-5,4,1],[-1,-4,5]]
//     mixed  Mq[c][a] = int phi_c psi_a   = (h/6) [[1,2,0],[0,2,1]]
//   with L_e = nu (M1 (x) K1 + K1 (x) M1), Bx_e = -(Mq (x) G),
//   By_e = -(G (x) Mq) (Kronecker order: y factor (x) x factor).
// * The 25 Vanka patch matrices of a level (paper, subsection "Vanka patch
//   matrices"), assembled locally from the elements around a representative
//   patch of each class, with the Dirichlet DoFs eliminated symmetrically,
//   and inverted once (the paper inverts the patch matrices ahead of time).
// * The coarsest-level operator, bordered by the constant-pressure vector
//   and inverted (Algorithm 1's exact level-0 solve).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "symmetry.h"
#include "mfma_patch.h"
#include <atomic>
#include <thread>

#include "vkmg_internal.h"

namespace vkmg {

namespace {

constexpr int K1n[3][3] = {{7, -8, 1}, {-8, 16, -8}, {1, -8, 7}};   // x 1/(3h)
constexpr int M1n[3][3] = {{4, 2, -1}, {2, 16, 2}, {-1, 2, 4}};     // x h/30
constexpr int Gn[2][3] = {{-5, 4, 1}, {-1, -4, 5}};                 // x 1/6
constexpr int Mqn[2][3] = {{1, 2, 0}, {0, 2, 1}};                   // x h/6

// Element Laplacian entry per unit viscosity between local Q2 nodes
// (a,b) and (c,d): (M1[b][d] K1[a][c] + K1[b][d] M1[a][c]), h-independent.
double elem_L(int a, int b, int c, int d) {
    return double(M1n[b][d] * K1n[a][c] + K1n[b][d] * M1n[a][c]) / 90.0;
}
// -int phi_(c,d) d psi_(a,b)/dx and /dy
double elem_Bx(int c, int d, int a, int b, double h) {
    return -h * double(Mqn[d][b] * Gn[c][a]) / 36.0;
}
double elem_By(int c, int d, int a, int b, double h) {
    return -h * double(Gn[d][b] * Mqn[c][a]) / 36.0;
}

}  // namespace

Geom make_geom(int32_t N, double nu) {
    Geom g;
    g.N = N;
    g.s2 = 2 * N + 1;
    g.s1 = N + 1;
    g.nq2 = int64_t(g.s2) * g.s2;
    g.nq1 = int64_t(g.s1) * g.s1;
    g.n = 2 * g.nq2 + g.nq1;
    g.h = 1.0 / double(N);
    g.nu = nu;
    return g;
}

int distance_class(int i, int N) {
    if (i == 0) return 0;
    if (i == N) return 4;
    if (i == 1) return 1;
    if (i == N - 1) return 3;
    return 2;
}

int class_representative(int c, int N) {
    switch (c) {
        case 0: return 0;
        case 1: return 1;
        case 2: return 2;
        case 3: return N - 1;
        default: return N;
    }
}

bool patch_matrix(int N, double nu, int cls, double* A, uint8_t* present) {
    if (N < 4 || cls < 0 || cls >= kClasses) return false;
    patch_matrix_at(N, nullptr, nu, class_representative(cls % 5, N),
                    class_representative(cls / 5, N), A, present);
    return true;
}

void patch_matrix_at(int N, const double* nu_elem, double nu, int I, int J, double* A,
                     uint8_t* present) {
    const double h = 1.0 / N;
    const int s2 = 2 * N + 1;
    std::fill(A, A + kSlots * kSlots, 0.0);
    uint8_t pres[kSlots];
    bool dir[kSlots];
    for (int b = 0; b < 5; ++b)
        for (int a = 0; a < 5; ++a) {
            const int qi = 2 * I - 2 + a, qj = 2 * J - 2 + b;
            const bool in = qi >= 0 && qi < s2 && qj >= 0 && qj < s2;
            const bool bnd = in && (qi == 0 || qj == 0 || qi == s2 - 1 || qj == s2 - 1);
            pres[5 * b + a] = pres[25 + 5 * b + a] = in ? 1 : 0;
            dir[5 * b + a] = dir[25 + 5 * b + a] = bnd;
        }
    pres[50] = 1;
    dir[50] = false;
    // slot of the Q2 node (qi, qj) or -1
    auto vslot = [&](int qi, int qj) -> int {
        const int a = qi - (2 * I - 2), b = qj - (2 * J - 2);
        if (a < 0 || a > 4 || b < 0 || b > 4) return -1;
        return 5 * b + a;
    };
    for (int ey = std::max(0, J - 2); ey <= std::min(N - 1, J + 1); ++ey)
        for (int ex = std::max(0, I - 2); ex <= std::min(N - 1, I + 1); ++ex) {
            int sl[9];
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) sl[3 * b + a] = vslot(2 * ex + a, 2 * ey + b);
            // pressure: only the patch's own Q1 node belongs to the patch
            int pl = -1;  // local Q1 index (d*2+c) of node (I,J) in this element
            for (int d = 0; d < 2; ++d)
                for (int c = 0; c < 2; ++c)
                    if (ex + c == I && ey + d == J) pl = 2 * d + c;
            const double nue = nu_elem ? nu_elem[int64_t(ey) * N + ex] : nu;
            for (int k = 0; k < 9; ++k) {
                if (sl[k] < 0) continue;
                const int a = k % 3, b = k / 3;
                for (int m = 0; m < 9; ++m) {
                    if (sl[m] < 0) continue;
                    const double v = nue * elem_L(a, b, m % 3, m / 3);
                    A[sl[k] * kSlots + sl[m]] += v;
                    A[(25 + sl[k]) * kSlots + 25 + sl[m]] += v;
                }
                if (pl >= 0) {
                    const int c = pl % 2, d = pl / 2;
                    const double bx = elem_Bx(c, d, a, b, h);
                    const double by = elem_By(c, d, a, b, h);
                    A[50 * kSlots + sl[k]] += bx;
                    A[sl[k] * kSlots + 50] += bx;
                    A[50 * kSlots + 25 + sl[k]] += by;
                    A[(25 + sl[k]) * kSlots + 50] += by;
                }
            }
        }
    // symmetric elimination of Dirichlet slots; identity on absent slots
    for (int s = 0; s < kSlots; ++s) {
        if (pres[s] && !dir[s]) continue;
        for (int t = 0; t < kSlots; ++t) {
            A[s * kSlots + t] = 0.0;
            A[t * kSlots + s] = 0.0;
        }
        A[s * kSlots + s] = 1.0;
    }
    if (present) std::memcpy(present, pres, kSlots);
}

bool invert_dense(int n, std::vector<double>& A, std::vector<double>& Ainv) {
    Ainv.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Ainv[size_t(i) * n + i] = 1.0;
    double scale = 0.0;
    for (double v : A) scale = std::max(scale, std::fabs(v));
    if (!(scale > 0.0) || !std::isfinite(scale)) return false;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = std::fabs(A[size_t(col) * n + col]);
        for (int r = col + 1; r < n; ++r) {
            const double v = std::fabs(A[size_t(r) * n + col]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        if (best <= 1e-13 * scale) return false;
        if (piv != col) {
            for (int c = 0; c < n; ++c) {
                std::swap(A[size_t(piv) * n + c], A[size_t(col) * n + c]);
                std::swap(Ainv[size_t(piv) * n + c], Ainv[size_t(col) * n + c]);
            }
        }
        const double d = 1.0 / A[size_t(col) * n + col];
        for (int c = 0; c < n; ++c) {
            A[size_t(col) * n + c] *= d;
            Ainv[size_t(col) * n + c] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = A[size_t(r) * n + col];
            if (f == 0.0) continue;
            double* ar = &A[size_t(r) * n];
            double* ir = &Ainv[size_t(r) * n];
            const double* ac = &A[size_t(col) * n];
            const double* ic = &Ainv[size_t(col) * n];
            for (int c = 0; c < n; ++c) {
                ar[c] -= f * ac[c];
                ir[c] -= f * ic[c];
            }
        }
    }
    return true;
}

void weighted_inverse(int N, int cls, double omega, const double* Ainv, const uint8_t* present,
                      double* W) {
    weighted_inverse_at(N, class_representative(cls % 5, N), class_representative(cls / 5, N),
                        omega, Ainv, present, W);
}

void weighted_inverse_at(int N, int I, int J, double omega, const double* Ainv,
                         const uint8_t* present, double* W) {
    const int s2 = 2 * N + 1;
    for (int s = 0; s < kSlots; ++s) {
        double w = 0.0;
        if (s == 50) {
            w = omega;  // each pressure DoF lies in exactly one patch
        } else if (present[s]) {
            const int loc = s % 25, a = loc % 5, b = loc / 5;
            const int qi = 2 * I - 2 + a, qj = 2 * J - 2 + b;
            const bool bnd = qi == 0 || qj == 0 || qi == s2 - 1 || qj == s2 - 1;
            if (!bnd) {
                // patches containing a free Q2 node: 3 per direction through a
                // vertex (even index), 2 through a midpoint (odd index)
                const int m = ((a % 2) ? 2 : 3) * ((b % 2) ? 2 : 3);
                w = omega / double(m);
            }
        }
        for (int t = 0; t < kSlots; ++t)
            W[s * kSlots + t] = (w != 0.0 && present[t]) ? w * Ainv[s * kSlots + t] : 0.0;
    }
}

void assemble_dense_level(int N, double nu, std::vector<double>& A, const double* nu_elem) {
    const Geom g = make_geom(N, nu);
    const int64_t n = g.n;
    A.assign(size_t(n) * n, 0.0);
    auto ux = [&](int qi, int qj) { return int64_t(qj) * g.s2 + qi; };
    auto uy = [&](int qi, int qj) { return g.nq2 + int64_t(qj) * g.s2 + qi; };
    auto pp = [&](int i, int j) { return 2 * g.nq2 + int64_t(j) * g.s1 + i; };
    for (int ey = 0; ey < N; ++ey)
        for (int ex = 0; ex < N; ++ex)
            for (int k = 0; k < 9; ++k) {
                const int a = k % 3, b = k / 3;
                const int qi = 2 * ex + a, qj = 2 * ey + b;
                const double nue = nu_elem ? nu_elem[int64_t(ey) * N + ex] : nu;
                for (int m = 0; m < 9; ++m) {
                    const int c = m % 3, d = m / 3;
                    const double v = nue * elem_L(a, b, c, d);
                    A[ux(qi, qj) * n + ux(2 * ex + c, 2 * ey + d)] += v;
                    A[uy(qi, qj) * n + uy(2 * ex + c, 2 * ey + d)] += v;
                }
                for (int l = 0; l < 4; ++l) {
                    const int c = l % 2, d = l / 2;
                    const int64_t P = pp(ex + c, ey + d);
                    const double bx = elem_Bx(c, d, a, b, g.h), by = elem_By(c, d, a, b, g.h);
                    A[P * n + ux(qi, qj)] += bx;
                    A[ux(qi, qj) * n + P] += bx;
                    A[P * n + uy(qi, qj)] += by;
                    A[uy(qi, qj) * n + P] += by;
                }
            }
    for (int qj = 0; qj < g.s2; ++qj)
        for (int qi = 0; qi < g.s2; ++qi) {
            if (!(qi == 0 || qj == 0 || qi == g.s2 - 1 || qj == g.s2 - 1)) continue;
            for (int64_t s : {ux(qi, qj), uy(qi, qj)}) {
                for (int64_t t = 0; t < n; ++t) {
                    A[s * n + t] = 0.0;
                    A[t * n + s] = 0.0;
                }
                A[s * n + s] = 1.0;
            }
        }
}

bool coarse_bordered_inverse(int N, double nu, std::vector<double>& C, const double* nu_elem) {
    const Geom g = make_geom(N, nu);
    const int64_t n = g.n, nb = n + 1;
    std::vector<double> A;
    assemble_dense_level(N, nu, A, nu_elem);
    std::vector<double> Ab(size_t(nb) * nb, 0.0);
    for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c < n; ++c) Ab[r * nb + c] = A[r * n + c];
    for (int64_t k = 2 * g.nq2; k < n; ++k) {
        Ab[k * nb + n] = 1.0;
        Ab[n * nb + k] = 1.0;
    }
    std::vector<double> inv;
    if (!invert_dense(int(nb), Ab, inv)) return false;
    C.assign(size_t(n) * n, 0.0);
    for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c < n; ++c) C[r * n + c] = inv[r * nb + c];
    return true;
}

bool interior_symmetry_blocks(const double* W, double* B, double tol) {
    // U = U1 (x) U1 per velocity component, identity on the pressure
    std::vector<double> U(kSlots * kSlots, 0.0);
    for (int f = 0; f < 2; ++f)
        for (int qb = 0; qb < 5; ++qb)
            for (int qa = 0; qa < 5; ++qa)
                for (int b = 0; b < 5; ++b)
                    for (int a = 0; a < 5; ++a)
                        U[(25 * f + 5 * qb + qa) * kSlots + 25 * f + 5 * b + a] =
                            double(sym_u1(qb, b) * sym_u1(qa, a));
    U[50 * kSlots + 50] = 1.0;
    double D[kSlots];
    for (int t = 0; t < kSlots; ++t) {
        double d = 0.0;
        for (int s = 0; s < kSlots; ++s) d += U[t * kSlots + s] * U[t * kSlots + s];
        D[t] = d;
    }
    // Bf = D^{-1} U W U^T D^{-1}
    std::vector<double> T1(kSlots * kSlots, 0.0), Bf(kSlots * kSlots, 0.0);
    for (int i = 0; i < kSlots; ++i)
        for (int k = 0; k < kSlots; ++k) {
            const double u = U[i * kSlots + k];
            if (u == 0.0) continue;
            for (int j = 0; j < kSlots; ++j) T1[i * kSlots + j] += u * W[k * kSlots + j];
        }
    double scale = 0.0;
    for (int i = 0; i < kSlots; ++i)
        for (int j = 0; j < kSlots; ++j) {
            double acc = 0.0;
            for (int k = 0; k < kSlots; ++k) acc += T1[i * kSlots + k] * U[j * kSlots + k];
            Bf[i * kSlots + j] = acc / (D[i] * D[j]);
            scale = std::max(scale, std::fabs(Bf[i * kSlots + j]));
        }
    for (int i = 0; i < kSlots; ++i)
        for (int j = 0; j < kSlots; ++j)
            if (sym_block_of(i) != sym_block_of(j) && std::fabs(Bf[i * kSlots + j]) > tol * scale)
                return false;
    for (int blk = 0; blk < kSymBlocks; ++blk) {
        const int n = sym_block_size(blk), off = sym_block_offset(blk);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                B[off + i * n + j] = Bf[sym_member(blk, i) * kSlots + sym_member(blk, j)];
    }
    return true;
}

bool universal_interior_blocks(double* B1) {
    const int N = 8;
    std::vector<double> A(kSlots * kSlots), inv;
    uint8_t pres[kSlots];
    if (!patch_matrix(N, 1.0, kInteriorClass, A.data(), pres)) return false;
    if (!invert_dense(kSlots, A, inv)) return false;
    // A1^{-1} = P8 A8^{-1} P8 with P8 = diag(I, 1/N): exact scalings by 2^-3
    for (int i = 0; i < kSlots; ++i)
        for (int j = 0; j < kSlots; ++j) {
            double f = 1.0;
            if (i == 50) f /= N;
            if (j == 50) f /= N;
            inv[i * kSlots + j] *= f;
        }
    std::vector<double> W(kSlots * kSlots);
    weighted_inverse(N, kInteriorClass, 1.0, inv.data(), pres, W.data());
    return interior_symmetry_blocks(W.data(), B1, 1e-12);
}

bool interior_d4_blocks(const double* B, double* C, double tol) {
    // full blocks in transformed coordinates: F[blk][i][j] = B at members i, j
    auto entry = [&](int blk, int tr, int tc) -> double {
        const int n = sym_block_size(blk), off = sym_block_offset(blk);
        int i = -1, j = -1;
        for (int k = 0; k < n; ++k) {
            if (sym_member(blk, k) == tr) i = k;
            if (sym_member(blk, k) == tc) j = k;
        }
        return (i < 0 || j < 0) ? 0.0 : B[off + i * n + j];
    };
    double scale = 0.0;
    for (int i = 0; i < kSymTotal; ++i) scale = std::max(scale, std::fabs(B[i]));
    const D4Table& d = kD4Table;
    // blocks 0 and 3: Q rows = [p], pair sums, pair differences; D = Q Q^T;
    // C = D^{-1} Q F Q^T D^{-1} must be even/odd block diagonal
    auto split = [&](int blk, const int* a, const int* b, bool with_p, double* Ce, double* Co) {
        const int np = 6, ne = np + (with_p ? 1 : 0), n = ne + np;
        std::vector<double> Q(size_t(n) * kSlots, 0.0), Dq(n, 0.0);
        int r = 0;
        if (with_p) Q[size_t(r++) * kSlots + 50] = 1.0;
        for (int k = 0; k < np; ++k, ++r) {
            Q[size_t(r) * kSlots + a[k]] = 1.0;
            Q[size_t(r) * kSlots + b[k]] = 1.0;
        }
        for (int k = 0; k < np; ++k, ++r) {
            Q[size_t(r) * kSlots + a[k]] = 1.0;
            Q[size_t(r) * kSlots + b[k]] = -1.0;
        }
        for (int i = 0; i < n; ++i)
            for (int t = 0; t < kSlots; ++t) Dq[i] += Q[size_t(i) * kSlots + t] * Q[size_t(i) * kSlots + t];
        std::vector<double> M(size_t(n) * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int t = 0; t < kSlots; ++t) {
                    const double qi = Q[size_t(i) * kSlots + t];
                    if (qi == 0.0) continue;
                    for (int u = 0; u < kSlots; ++u) {
                        const double qj = Q[size_t(j) * kSlots + u];
                        if (qj != 0.0) acc += qi * entry(blk, t, u) * qj;
                    }
                }
                M[size_t(i) * n + j] = acc / (Dq[i] * Dq[j]);
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const bool same = (i < ne) == (j < ne);
                if (!same && std::fabs(M[size_t(i) * n + j]) > tol * scale) return false;
            }
        for (int i = 0; i < ne; ++i)
            for (int j = 0; j < ne; ++j) Ce[i * ne + j] = M[size_t(i) * n + j];
        for (int i = 0; i < np; ++i)
            for (int j = 0; j < np; ++j) Co[i * np + j] = M[size_t(ne + i) * n + ne + j];
        return true;
    };
    if (!split(0, d.a0, d.b0, true, C + kD4Off0e, C + kD4Off0o)) return false;
    if (!split(3, d.a3, d.b3, false, C + kD4Off3e, C + kD4Off3o)) return false;
    // blocks 1 and 2: block 2 is block 1 relabelled by the reflection
    for (int i = 0; i < 13; ++i)
        for (int k = 0; k < 13; ++k) {
            const double c1 = entry(1, d.m1[i], d.m1[k]);
            const double c2 = entry(2, d.m2[i], d.m2[k]);
            if (std::fabs(c1 - c2) > tol * scale) return false;
            C[kD4Off1 + i * 13 + k] = c1;
        }
    return true;
}

void mfma_interior_table(const double* B1, bool fp64_layout, double* A) {
    // member index of transformed slot t within its block
    int member[kSlots];
    for (int blk = 0; blk < kSymBlocks; ++blk)
        for (int k = 0; k < sym_block_size(blk); ++k) member[sym_member(blk, k)] = k;
    for (int blk = 0; blk < kSymBlocks; ++blk) {
        const int n = sym_block_size(blk), off = sym_block_offset(blk);
        for (int c = 0; c < 4; ++c)
            for (int lane = 0; lane < 64; ++lane) {
                const int i = lane % 16, k = lane / 16;
                // output row i sits in quarter i / 4, element i % 4 (FP32)
                // or in quarter i % 4, element i / 4 (FP64)
                const int qr = fp64_layout ? i % 4 : i / 4, vr = fp64_layout ? i / 4 : i % 4;
                const int tr = quarter_item_tslot(blk, qr, vr);
                const int tc = quarter_item_tslot(blk, k, c);
                double v = 0.0;
                if (tr >= 0 && tc >= 0) v = B1[off + member[tr] * n + member[tc]];
                A[(blk * 4 + c) * 64 + lane] = v;
            }
    }
}

double universal_mismatch(const double* Blevel, const double* B1, double omega, double nu,
                          double h) {
    const double scale = omega / nu, t = nu / h;
    double err = 0.0, ref = 0.0;
    for (int blk = 0; blk < kSymBlocks; ++blk) {
        const int n = sym_block_size(blk), off = sym_block_offset(blk);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double f = scale;
                if (sym_member(blk, i) == 50) f *= t;
                if (sym_member(blk, j) == 50) f *= t;
                const double want = f * B1[off + i * n + j];
                err = std::max(err, std::fabs(Blevel[off + i * n + j] - want));
                ref = std::max(ref, std::fabs(Blevel[off + i * n + j]));
            }
    }
    return err / ref;
}

// Weighted inverses of every patch of an N x N level with per-element
// viscosity nu_elem (N^2 values, index ey*N + ex), each stored transposed
// (51 x 51, column s of W_i at [s*51, s*51+51)) at out + k*51*51 for patch
// k = J*(N+1) + I; patches are split over the host threads.  Returns false
// if a patch matrix is singular.
bool simple_vanka_tables(int N, const double* nu_elem, double omega, double* out) {
    const int P = (N + 1) * (N + 1);
    unsigned nt = std::thread::hardware_concurrency();
    if (nt < 1) nt = 1;
    if (nt > 64) nt = 64;
    std::atomic<bool> ok{true};
    auto work = [&](int t) {
        std::vector<double> A(kSlots * kSlots), inv, W(kSlots * kSlots);
        uint8_t pres[kSlots];
        for (int k = t; k < P && ok.load(); k += int(nt)) {
            const int I = k % (N + 1), J = k / (N + 1);
            patch_matrix_at(N, nu_elem, 1.0, I, J, A.data(), pres);
            if (!invert_dense(kSlots, A, inv)) {
                ok = false;
                return;
            }
            weighted_inverse_at(N, I, J, omega, inv.data(), pres, W.data());
            double* o = out + int64_t(k) * kSlots * kSlots;
            for (int i = 0; i < kSlots; ++i)
                for (int j = 0; j < kSlots; ++j) o[j * kSlots + i] = W[i * kSlots + j];
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(work, int(t));
    for (auto& x : th) x.join();
    return ok.load();
}

}  // namespace vkmg
