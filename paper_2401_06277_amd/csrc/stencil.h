// Matrix-free rows of the Q2-Q1 Stokes operator on a uniform mesh.
//
// The assembled operator of the paper's equation "stokesmatrix" is a tensor
// product of 1D assembled factors (rows indexed by node parity: 0 = mesh
// vertex, even Q2 index; 1 = element midpoint, odd Q2 index; entries by the
// offset -2..2 of the column node):
//   stiffness K (x 1/(3h)): vertex [1,-8,14,-8,1], midpoint [0,-8,16,-8,0]
//   mass      M (x h/30)  : vertex [-1,2,8,2,-1], midpoint [0,2,16,2,0]
// and, for a Q1 row I against Q2 column i with offset o = i - 2I,
//   G  = int phi_I psi_i'  (x 1/6) : [-1,-4,0,4,1]
//   Mq = int phi_I psi_i   (x h/6) : [0,2,2,2,0]
// so that, with L = M (x) K + K (x) M (per velocity component, times nu) and
// B = [-(Mq (x) G), -(G (x) Mq)]:
//   (L u)(i,j)     = nu/90  sum_{dx,dy} (M[py][dy] K[px][dx] + K[py][dy] M[px][dx]) u(i+dx, j+dy)
//   (B u)(I,J)     = -h/36  sum_{ox,oy} (Mq[oy] G[ox] u_x + G[oy] Mq[ox] u_y)(2I+ox, 2J+oy)
//   (B^T p)_x(i,j) = -h/36  sum_{I,J} Mq[j-2J] G[i-2I] p(I,J)   (u_y: G and Mq swapped)
// These interior formulas also give the rows of Q1 nodes on the boundary
// and of free Q2 nodes next to it, once velocity values on the boundary
// (Dirichlet columns) and outside the domain are read as zero.  All integer
// numerators are exact, so structural zeros (e.g. midpoint-to-midpoint two
// nodes apart) fold away at compile time.
#pragma once

#include <hip/hip_runtime.h>

namespace vkmg {

__host__ __device__ constexpr int st_K(int par, int o) {
    return par == 0 ? (o == 0 ? 14 : (o == 1 || o == -1) ? -8 : 1)
                    : (o == 0 ? 16 : (o == 1 || o == -1) ? -8 : 0);
}
__host__ __device__ constexpr int st_M(int par, int o) {
    return par == 0 ? (o == 0 ? 8 : (o == 1 || o == -1) ? 2 : -1)
                    : (o == 0 ? 16 : (o == 1 || o == -1) ? 2 : 0);
}
__host__ __device__ constexpr int st_L(int py, int px, int dy, int dx) {
    return st_M(py, dy) * st_K(px, dx) + st_K(py, dy) * st_M(px, dx);
}
__host__ __device__ constexpr int st_G(int o) {
    return o == -2 ? -1 : o == -1 ? -4 : o == 0 ? 0 : o == 1 ? 4 : 1;
}
__host__ __device__ constexpr int st_Mq(int o) { return (o == -2 || o == 2) ? 0 : 2; }

// The same Q1-row factors for a row I that may lie on the boundary (I == 0
// or I == N), where only one element contributes.  Needed when boundary
// velocity values are read (the Dirichlet lifting), not when they are
// masked.
__host__ __device__ constexpr int st_G_row(int I, int N, int o) {
    return I == 0 ? (o == 0 ? -5 : o == 1 ? 4 : o == 2 ? 1 : 0)
         : I == N ? (o == -2 ? -1 : o == -1 ? -4 : o == 0 ? 5 : 0)
                  : st_G(o);
}
__host__ __device__ constexpr int st_Mq_row(int I, int N, int o) {
    return I == 0 ? (o == 0 ? 1 : o == 1 ? 2 : 0)
         : I == N ? (o == 0 ? 1 : o == -1 ? 2 : 0)
                  : st_Mq(o);
}

}  // namespace vkmg
