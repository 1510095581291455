// Build-time generator of the universal interior Vanka operator.
//
// On a uniform mesh the interior patch matrix of the level with mesh size h
// and viscosity nu is A = P A1 P with P = diag(sqrt(nu) I_vel, h/sqrt(nu))
// and A1 the interior patch matrix for h = nu = 1 (L is h-independent in
// 2D, B is proportional to h).  Hence the weighted inverse is
//   W = omega diag(1/m) A^{-1} = (omega/nu) D W1 D,  D = diag(I_vel, nu/h),
// with W1 = diag(1/m) A1^{-1} universal.  This program assembles the
// interior patch on an 8 x 8 mesh (nu = 1), removes the exact power-of-two
// scaling of its pressure row and column, splits W1 by the symmetries of
// the square (symmetry.h), checks the split form against the plain
// reflection blocks on random vectors, and prints its 326 constants as a
// header.
#include <cmath>
#include <cstdio>
#include <random>

#include "d4_apply.h"
#include "symmetry.h"
#include "vkmg_internal.h"

using namespace vkmg;

int main() {
    double B[kSymTotal], C[kD4Total];
    if (!universal_interior_blocks(B)) return 1;
    if (!interior_d4_blocks(B, C, 1e-12)) {
        std::fprintf(stderr, "interior operator does not have the dihedral block structure\n");
        return 2;
    }
    // check: d4_apply against U^T (reflection blocks) U on random vectors
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> uni(-1.0, 1.0);
    double err = 0.0, ref = 0.0;
    for (int trial = 0; trial < 16; ++trial) {
        double v[51], w[51];
        for (int s = 0; s < 51; ++s) v[s] = w[s] = uni(rng);
        const double t = 1.0 + trial;
        w[50] *= t;  // the caller's input scaling of the pressure
        v[50] *= t;
        d4_apply(v, t, [&](int i) { return C[i]; });
        // reference: forward butterflies, reflection blocks, transpose
        for (int f = 0; f < 2; ++f) {
            for (int b = 0; b < 5; ++b) d4_bfly(w, 25 * f + 5 * b, 1);
            for (int q = 0; q < 5; ++q) d4_bfly(w, 25 * f + q, 5);
        }
        double y[51] = {0};
        for (int blk = 0; blk < kSymBlocks; ++blk) {
            const int n = sym_block_size(blk), off = sym_block_offset(blk);
            for (int i = 0; i < n; ++i) {
                double acc = 0.0;
                for (int j = 0; j < n; ++j) acc += B[off + i * n + j] * w[sym_member(blk, j)];
                y[sym_member(blk, i)] = acc;
            }
        }
        y[50] *= t;
        for (int f = 0; f < 2; ++f) {
            for (int q = 0; q < 5; ++q) d4_bfly_t(y, 25 * f + q, 5);
            for (int b = 0; b < 5; ++b) d4_bfly_t(y, 25 * f + 5 * b, 1);
        }
        for (int s = 0; s < 51; ++s) {
            err = std::fmax(err, std::fabs(v[s] - y[s]));
            ref = std::fmax(ref, std::fabs(y[s]));
        }
    }
    if (!(err <= 1e-12 * ref)) {
        std::fprintf(stderr, "dihedral apply differs from the reflection blocks: %g of %g\n", err, ref);
        return 3;
    }
    std::printf("// Generated at build time by gen_interior_blocks.cpp; do not edit.\n");
    std::printf("// Universal interior weighted inverse W1 = diag(1/m) A1^{-1} (mesh size 1,\n");
    std::printf("// unit viscosity) in the dihedral coordinates of symmetry.h (kD4Off* layout).\n");
    std::printf("#pragma once\nnamespace vkmg {\n");
    std::printf("__device__ constexpr double kInteriorD4[%d] = {\n", kD4Total);
    for (int i = 0; i < kD4Total; ++i) std::printf("    %.17g,\n", C[i]);
    std::printf("};\n}  // namespace vkmg\n");
    return 0;
}
