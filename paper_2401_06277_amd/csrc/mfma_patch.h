// Interior Vanka patch apply on the 16x16x4 matrix instructions.
//
// The interior operator is block diagonal in the reflection-adapted
// coordinates of symmetry.h (blocks of 13, 13, 13 and 12).  Each block is
// applied to 16 patches at once as a 16x16 (padded) matrix times a 16 x 16
// matrix of patch vectors, four K=4 steps per block, 16 instructions for
// 16 patches.  Lane l of a wave serves patch j = l % 16 of the current row
// of 16 patches and quarter q = l / 16 of its slots.
//
// Operand layout of the 16x16x4 instructions: A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k; D[i][j] in element r of lane j + 16 q with
// i = 4q + r for FP32 and i = 4r + q for FP64 (checked on the device).  So
// in step c the K index is the lane quarter q, and element v of quarter q
// holds one output row (4q + v or 4v + q).  Both the input position (q, c)
// and the output position (q, v) are chosen to be "item v (or c) of
// quarter q" (the operand table orders the rows accordingly), with the
// items of a quarter being
//   item 0, 1: the full reflection orbit (a = item, b = q & 1) of component
//              q >> 1 (u_x for q < 2, u_y for q >= 2): the four slots
//              (a, b), (4-a, b), (a, 4-b), (4-a, 4-b), whose four
//              transformed values lie in the four different blocks;
//   item 2:    a pair of half orbits, u_x and u_y about the x centre line
//              (slots (2, b), (2, 4-b), b = q) for q < 2, about the y
//              centre line (slots (a, 2), (4-a, 2), a = q - 2) for q >= 2;
//              again one transformed value per block;
//   item 3:    for q = 0 the three fixed slots p, u_x(2,2), u_y(2,2)
//              (blocks 0, 1, 2); padding otherwise.
// Every slot of the patch is in exactly one item, so the butterflies of
// symmetry.h (forward U and transposed U^T) are lane-local: a quarter reads
// 15 raw residual values (the last three only matter for q = 0) and
// produces 15 raw corrections in the same order.
//
// Block of each transformed value (symmetry.h sym_block_of), with ss, ds,
// sd, dd the sum/difference combinations in x and y of a full orbit:
//   u_x: ss -> 1, ds -> 0, sd -> 3, dd -> 2;  u_y: ss -> 2, ds -> 3,
//   sd -> 0, dd -> 1.  The u_y case equals the u_x formulas applied with
//   the two mixed raw values negated (sign s = -1), and on output with the
//   two mixed results negated.
#pragma once

#include "symmetry.h"

namespace vkmg {

constexpr int kQuarterValues = 15;

// Patch slot (0..50) of value k (0..14) of quarter q.
constexpr int quarter_slot(int q, int k) {
    const int f = q >> 1, b = q & 1;
    const int off = 25 * f;
    if (k < 8) {
        const int a = k >> 2;  // full orbit item 0 (a = 0) or 1 (a = 1)
        const int m = k & 3;   // (a, b), (4-a, b), (a, 4-b), (4-a, 4-b)
        const int aa = (m & 1) ? 4 - a : a;
        const int bb = (m & 2) ? 4 - b : b;
        return off + 5 * bb + aa;
    }
    if (k < 12) {
        const int m = k - 8;  // u_x first/second, u_y first/second
        const int fo = (m >> 1) * 25;
        if (q < 2) {
            const int bb = (m & 1) ? 4 - q : q;
            return fo + 5 * bb + 2;
        }
        const int a = q - 2;
        const int aa = (m & 1) ? 4 - a : a;
        return fo + 10 + aa;
    }
    return k == 12 ? 50 : k == 13 ? 12 : 37;
}

// Transformed slot (symmetry.h numbering) of item v of quarter q in block
// blk, or -1 if the item has no value in that block (padding).
constexpr int quarter_item_tslot(int blk, int q, int v) {
    int cand[4] = {-1, -1, -1, -1};
    if (v < 2) {
        const int f = q >> 1, b = q & 1, a = v;
        cand[0] = 25 * f + 5 * b + a;              // ss
        cand[1] = 25 * f + 5 * b + 3 + a;          // ds
        cand[2] = 25 * f + 5 * (3 + b) + a;        // sd
        cand[3] = 25 * f + 5 * (3 + b) + 3 + a;    // dd
    } else if (v == 2) {
        if (q < 2) {
            const int b = q;
            cand[0] = 5 * b + 2;
            cand[1] = 5 * (3 + b) + 2;
            cand[2] = 25 + 5 * b + 2;
            cand[3] = 25 + 5 * (3 + b) + 2;
        } else {
            const int a = q - 2;
            cand[0] = 10 + a;
            cand[1] = 10 + 3 + a;
            cand[2] = 35 + a;
            cand[3] = 35 + 3 + a;
        }
    } else if (q == 0) {
        cand[0] = 50;
        cand[1] = 12;
        cand[2] = 37;
    }
    for (int i = 0; i < 4; ++i)
        if (cand[i] >= 0 && sym_block_of(cand[i]) == blk) return cand[i];
    return -1;
}

// Forward transform of one quarter: raw values in[15] (residual slots in
// quarter_slot order) -> B[blk][c], the value of item c in block blk.
template <typename T>
constexpr void quarter_forward(int q, const T (&in)[kQuarterValues], T (&B)[4][4]) {
    const T s = q < 2 ? T(1) : T(-1);
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        const T v00 = in[4 * o], v10 = in[4 * o + 1], v01 = in[4 * o + 2], v11 = in[4 * o + 3];
        const T X = v00 + s * v10, Xd = v00 - s * v10;
        const T Y = s * v01 + v11, Yd = s * v01 - v11;
        B[0][o] = Xd + Yd;
        B[1][o] = X + Y;
        B[2][o] = Xd - Yd;
        B[3][o] = X - Y;
    }
    const T sx = in[8] + in[9], dx = in[8] - in[9];
    const T sy = in[10] + in[11], dy = in[10] - in[11];
    B[0][2] = q < 2 ? dy : dx;
    B[1][2] = sx;
    B[2][2] = sy;
    B[3][2] = q < 2 ? dx : dy;
    B[0][3] = in[12];
    B[1][3] = in[13];
    B[2][3] = in[14];
    B[3][3] = T(0);
}

// Inverse (transposed) transform of one quarter: D[blk][v], the block
// outputs of item v -> raw corrections out[15] in quarter_slot order.  The
// pressure output is multiplied by t (the D = diag(I, t) scaling).
template <typename T>
constexpr void quarter_inverse(int q, const T (&D)[4][4], T t, T (&out)[kQuarterValues]) {
    const T s = q < 2 ? T(1) : T(-1);
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        const T y0 = D[0][o], y1 = D[1][o], y2 = D[2][o], y3 = D[3][o];
        const T P = y0 + y1, Q = y1 - y0, R = y2 + y3, S = y3 - y2;
        out[4 * o] = P + R;
        out[4 * o + 1] = s * (Q + S);
        out[4 * o + 2] = s * (P - R);
        out[4 * o + 3] = Q - S;
    }
    const T m1 = q < 2 ? D[3][2] : D[0][2];
    const T m2 = q < 2 ? D[0][2] : D[3][2];
    out[8] = D[1][2] + m1;
    out[9] = D[1][2] - m1;
    out[10] = D[2][2] + m2;
    out[11] = D[2][2] - m2;
    out[12] = t * D[0][3];
    out[13] = D[1][3];
    out[14] = D[2][3];
}

}  // namespace vkmg
