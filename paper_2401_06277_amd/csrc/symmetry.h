// Reflection-adapted coordinates of an interior Vanka patch.
//
// An interior patch (pressure node two or more elements from the boundary)
// is mapped onto itself by the reflections x -> 2x_c - x and y -> 2y_c - y
// about its pressure node.  The Stokes operator is invariant under them
// when the reflected velocity component changes sign, so the patch matrix,
// its inverse and the weighted inverse W A^{-1} (the weights 1/m_j are
// reflection invariant) commute with the signed permutations
//   sigma_x: u_x(a,b) -> -u_x(4-a,b), u_y(a,b) -> u_y(4-a,b), p -> p
//   sigma_y: u_x(a,b) -> u_x(a,4-b), u_y(a,b) -> -u_y(a,4-b), p -> p
// (a, b = 0..4 the node of the 5x5 patch grid).  In coordinates that are
// even or odd under each reflection the matrix is block diagonal, one block
// per pair of eigenvalues (+-1, +-1) of (sigma_x, sigma_y), of sizes
// 13, 13, 13, 12.
//
// Transform (per velocity component, on the 5x5 grid, separable):
//   1D forward  U1: (f0,f1,f2,f3,f4) -> (f0+f4, f1+f3, f2, f0-f4, f1-f3)
//   2D          U = U1 (x) U1 (y factor (x) x factor), transformed index
//               5*qb + qa; p is left as is.
// U U^T = D is diagonal, U^{-1} = U^T D^{-1}, and for any M commuting with
// the reflections  M r = U^T (B (U r))  with  B = D^{-1} U M U^T D^{-1}
// block diagonal.  Only additions are needed for U and U^T.
//
// Transformed slot t: 25*f + 5*qb + qa for velocity component f (0: u_x,
// 1: u_y), 50 for the pressure.  Plain constexpr functions, usable from
// host and device code.
#pragma once

namespace vkmg {

constexpr int kSymBlocks = 4;
constexpr int kSymTotal = 13 * 13 * 3 + 12 * 12;  // 651

// Block of transformed slot t: (sigma_x eigenvalue < 0) + 2 (sigma_y eigenvalue < 0).
constexpr int sym_block_of(int t) {
    if (t == 50) return 0;
    const int f = t / 25, q = t % 25, qa = q % 5, qb = q / 5;
    const bool xodd = qa >= 3, yodd = qb >= 3;
    // a coordinate odd in x is even under sigma_x for u_x (sign flip) and
    // odd for u_y; likewise in y with the roles of the components swapped
    const bool sx_neg = (f == 0) ? !xodd : xodd;
    const bool sy_neg = (f == 0) ? yodd : !yodd;
    return (sx_neg ? 1 : 0) + (sy_neg ? 2 : 0);
}

constexpr int sym_block_size(int blk) { return blk == 3 ? 12 : 13; }

constexpr int sym_block_offset(int blk) {
    return blk == 0 ? 0 : blk == 1 ? 169 : blk == 2 ? 338 : 507;
}

// k-th transformed slot (increasing t) of block blk.
constexpr int sym_member(int blk, int k) {
    int c = 0;
    for (int t = 0; t < 51; ++t) {
        if (sym_block_of(t) == blk) {
            if (c == k) return t;
            ++c;
        }
    }
    return -1;
}

// Member table, built at compile time so that device code indexes it with
// constants after unrolling.
struct SymTable {
    int m[kSymBlocks][13];
};
constexpr SymTable make_sym_table() {
    SymTable t{};
    for (int blk = 0; blk < kSymBlocks; ++blk)
        for (int k = 0; k < 13; ++k) t.m[blk][k] = k < sym_block_size(blk) ? sym_member(blk, k) : 0;
    return t;
}
constexpr SymTable kSymTable = make_sym_table();

// Diagonal reflection (x, y) -> (y, x) about the patch node.  It maps
// u_x(a, b) -> u_y(b, a), u_y(a, b) -> u_x(b, a), p -> p, so in the
// transformed coordinates (U1 is the same in x and y) t = 25 f + 5 qb + qa
// goes to 25 (1 - f) + 5 qa + qb, a plain permutation.  It swaps blocks 1
// and 2 and maps blocks 0 and 3 onto themselves; the interior operator
// commutes with it, so
//   * block 2 is block 1 with rows and columns relabelled by the
//     reflection (one set of constants serves both), and
//   * blocks 0 and 3 split further into reflection-even coordinates
//     (x_t + x_dt for the pairs t < dt, and p) and reflection-odd ones
//     (x_t - x_dt): 13 = 7 + 6 and 12 = 6 + 6.
// Together with the x/y reflections this is the dihedral group of the
// square; 7^2 + 6^2 + 13^2 + 6^2 + 6^2 = 326 constants and 49 + 36 + 2 x
// 169 + 36 + 36 = 495 multiply-adds per patch.
constexpr int sym_delta(int t) {
    if (t == 50) return 50;
    const int f = t / 25, q = t % 25;
    return 25 * (1 - f) + 5 * (q % 5) + q / 5;
}

constexpr int kD4Total = 7 * 7 + 6 * 6 + 13 * 13 + 6 * 6 + 6 * 6;  // 326
// offsets of the D4 blocks: 0-even (7), 0-odd (6), 1 (13, shared by 2),
// 3-even (6), 3-odd (6)
constexpr int kD4Off0e = 0, kD4Off0o = 49, kD4Off1 = 85, kD4Off3e = 254, kD4Off3o = 290;

struct D4Table {
    int a0[6], b0[6];  // block-0 pairs (a < b = delta(a)), increasing a
    int a3[6], b3[6];  // block-3 pairs
    int m1[13], m2[13];  // block-1 members and their images in block 2
};
constexpr D4Table make_d4_table() {
    D4Table d{};
    int n0 = 0, n3 = 0, n1 = 0;
    for (int t = 0; t < 50; ++t) {
        const int u = sym_delta(t);
        const int blk = sym_block_of(t);
        if (blk == 0 && t < u) {
            d.a0[n0] = t;
            d.b0[n0] = u;
            ++n0;
        } else if (blk == 3 && t < u) {
            d.a3[n3] = t;
            d.b3[n3] = u;
            ++n3;
        } else if (blk == 1) {
            d.m1[n1] = t;
            d.m2[n1] = u;
            ++n1;
        }
    }
    return d;
}
constexpr D4Table kD4Table = make_d4_table();

// Entry (row qa/qb, column a/b) of the 1D forward transform U1.
constexpr int sym_u1(int q, int a) {
    return q == 0 ? ((a == 0 || a == 4) ? 1 : 0)
         : q == 1 ? ((a == 1 || a == 3) ? 1 : 0)
         : q == 2 ? (a == 2 ? 1 : 0)
         : q == 3 ? (a == 0 ? 1 : a == 4 ? -1 : 0)
                  : (a == 1 ? 1 : a == 3 ? -1 : 0);
}

}  // namespace vkmg
