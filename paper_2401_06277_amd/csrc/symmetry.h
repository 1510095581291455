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

// Entry (row qa/qb, column a/b) of the 1D forward transform U1.
constexpr int sym_u1(int q, int a) {
    return q == 0 ? ((a == 0 || a == 4) ? 1 : 0)
         : q == 1 ? ((a == 1 || a == 3) ? 1 : 0)
         : q == 2 ? (a == 2 ? 1 : 0)
         : q == 3 ? (a == 0 ? 1 : a == 4 ? -1 : 0)
                  : (a == 1 ? 1 : a == 3 ? -1 : 0);
}

}  // namespace vkmg
