// Interior Vanka operator applied in the coordinates of the symmetry group
// of the square (symmetry.h): reflection butterflies in x and y, then the
// diagonal-reflection split of blocks 0 and 3 and the shared constants of
// blocks 1 and 2, then the transposed butterflies.
//
//   v <- D W1 D v,  D = diag(I, t) (the pressure output is scaled by t here;
//   the caller scales the input).
//
// `coef(i)` returns constant i of the 326-value table (symmetry.h kD4Off*
// layout).  The same code runs on the device with compile-time constants
// and on the host (build-time check) with a runtime table.
#pragma once

#include "symmetry.h"

namespace vkmg {

// 1D reflection butterfly and its transpose on 5 values v[o + k*st].
template <typename T, int N>
constexpr void d4_bfly(T (&v)[N], int o, int st) {
    const T f0 = v[o], f1 = v[o + st], f3 = v[o + 3 * st], f4 = v[o + 4 * st];
    v[o] = f0 + f4;
    v[o + st] = f1 + f3;
    v[o + 3 * st] = f0 - f4;
    v[o + 4 * st] = f1 - f3;
}
template <typename T, int N>
constexpr void d4_bfly_t(T (&v)[N], int o, int st) {
    const T e0 = v[o], e1 = v[o + st], o0 = v[o + 3 * st], o1 = v[o + 4 * st];
    v[o] = e0 + o0;
    v[o + st] = e1 + o1;
    v[o + 3 * st] = e1 - o1;
    v[o + 4 * st] = e0 - o0;
}

// y = C x for an n x n block of the table at offset off (two partial sums
// per row for instruction-level parallelism).
template <typename T, int NN, typename Coef>
constexpr void d4_block(const T (&x)[NN], T (&y)[NN], int off, Coef coef) {
#pragma unroll
    for (int i = 0; i < NN; ++i) {
        T a0 = 0, a1 = 0;
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            const T c = T(coef(off + i * NN + j));
            if (j & 1)
                a1 += c * x[j];
            else
                a0 += c * x[j];
        }
        y[i] = a0 + a1;
    }
}

template <typename T, typename Coef>
constexpr void d4_apply(T (&v)[51], T t, Coef coef) {
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int b = 0; b < 5; ++b) d4_bfly(v, 25 * f + 5 * b, 1);
#pragma unroll
        for (int q = 0; q < 5; ++q) d4_bfly(v, 25 * f + q, 5);
    }
    const D4Table& d = kD4Table;
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
    // blocks 1 and 2: one set of constants, each used twice
    {
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
            v[d.m1[i]] = y1[i];
            v[d.m2[i]] = y2[i];
        }
    }
    v[50] *= t;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int q = 0; q < 5; ++q) d4_bfly_t(v, 25 * f + q, 5);
#pragma unroll
        for (int b = 0; b < 5; ++b) d4_bfly_t(v, 25 * f + 5 * b, 1);
    }
}

}  // namespace vkmg
