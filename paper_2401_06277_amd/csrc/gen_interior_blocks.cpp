// Build-time generator of the universal interior Vanka operator.
//
// On a uniform mesh the interior patch matrix of the level with mesh size h
// and viscosity nu is A = P A1 P with P = diag(sqrt(nu) I_vel, h/sqrt(nu))
// and A1 the interior patch matrix for h = nu = 1 (L is h-independent in
// 2D, B is proportional to h).  Hence the weighted inverse is
//   W = omega diag(1/m) A^{-1} = (omega/nu) D W1 D,  D = diag(I_vel, nu/h),
// with W1 = diag(1/m) A1^{-1} universal.  This program assembles the
// interior patch on an 8 x 8 mesh (nu = 1), removes the exact power-of-two
// scaling of its pressure row and column, and prints the reflection blocks
// of W1 (symmetry.h) as a header of compile-time constants.
#include <cstdio>

#include "symmetry.h"
#include "vkmg_internal.h"

using namespace vkmg;

int main() {
    double B[kSymTotal];
    if (!universal_interior_blocks(B)) return 1;
    std::printf("// Generated at build time by gen_interior_blocks.cpp; do not edit.\n");
    std::printf("// Reflection blocks (symmetry.h) of the universal interior weighted\n");
    std::printf("// inverse W1 = diag(1/m) A1^{-1} for mesh size 1 and unit viscosity.\n");
    std::printf("#pragma once\nnamespace vkmg {\n");
    std::printf("__device__ constexpr double kInteriorW1[%d] = {\n", kSymTotal);
    for (int i = 0; i < kSymTotal; ++i) std::printf("    %.17g,\n", B[i]);
    std::printf("};\n}  // namespace vkmg\n");
    return 0;
}
