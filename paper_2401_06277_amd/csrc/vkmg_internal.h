// Internal declarations shared by the host setup code, the kernels and the
// C-ABI layer of the vkmg library.  Not part of the public interface.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace vkmg {

constexpr int kSlots = 51;    // DoFs of a full Vanka patch: 2 x 25 velocity + 1 pressure
constexpr int kClasses = 25;  // distinct patch matrices on a uniform mesh
constexpr int kInteriorClass = 12;  // class_x = class_y = 2

// Geometry of one level (N elements per side).
struct Geom {
    int32_t N;       // elements per side
    int32_t s2, s1;  // Q2 and Q1 nodes per side: 2N+1, N+1
    int64_t nq2;     // (2N+1)^2
    int64_t nq1;     // (N+1)^2
    int64_t n;       // 2 nq2 + nq1
    double h;        // 1/N
    double nu;       // viscosity
};

Geom make_geom(int32_t N, double nu);

// ---------------------------------------------------------------------------
// Host setup (host_setup.cpp), pure C++ in FP64.
// ---------------------------------------------------------------------------

// 0: low boundary, 1: one element in, 2: interior, 3: one element from the
// high boundary, 4: high boundary.  Requires N >= 4 for five distinct classes.
int distance_class(int i, int N);
int class_representative(int c, int N);

// Patch matrix of class `cls` (51x51 row-major, absent slots identity).
// Returns false if the arguments are out of range.
bool patch_matrix(int N, double nu, int cls, double* A, uint8_t* present);
// Patch matrix of the patch at Q1 node (I, J); per-element viscosity
// nu_elem (N^2 values, index ey*N + ex) or, if NULL, the constant nu.
void patch_matrix_at(int N, const double* nu_elem, double nu, int I, int J, double* A,
                     uint8_t* present);

// In-place Gauss-Jordan inversion with partial pivoting; false if singular.
bool invert_dense(int n, std::vector<double>& A, std::vector<double>& Ainv);

// Weighted inverse W A^{-1}: row s scaled by omega/m_s for present free
// slots, zero for Dirichlet and absent slots.
void weighted_inverse(int N, int cls, double omega, const double* Ainv, const uint8_t* present,
                      double* W);
void weighted_inverse_at(int N, int I, int J, double omega, const double* Ainv,
                         const uint8_t* present, double* W);
// Transposed weighted inverses of all (N+1)^2 patches for a per-element
// viscosity (51*51 values per patch, patch k = J*(N+1) + I); false if a
// patch matrix is singular.
bool simple_vanka_tables(int N, const double* nu_elem, double omega, double* out);

// Dense constrained operator of the whole level (n x n, row-major).
void assemble_dense_level(int N, double nu, std::vector<double>& A,
                          const double* nu_elem = nullptr);

// Top-left n x n block of the inverse of the matrix bordered by the
// constant-pressure vector; false if singular.
bool coarse_bordered_inverse(int N, double nu, std::vector<double>& C,
                             const double* nu_elem = nullptr);

// Block-diagonal form of the interior weighted inverse W in the reflection-
// adapted coordinates of symmetry.h (651 values, blocks concatenated
// row-major).  Returns false if W does not commute with the reflections to
// within `tol` relative to its largest entry.
bool interior_symmetry_blocks(const double* W, double* B, double tol);

// Reflection blocks of the universal interior operator W1 (mesh size 1,
// unit viscosity, unit damping); the operator of a level with mesh size h,
// viscosity nu and damping omega is (omega/nu) D W1 D, D = diag(I, nu/h).
bool universal_interior_blocks(double* B1);
// Largest deviation of a level's blocks from that scaled universal form,
// relative to the largest block entry.
double universal_mismatch(const double* Blevel, const double* B1, double omega, double nu,
                          double h);

// The reflection blocks (651 values) refined by the diagonal reflection
// (symmetry.h kD4Table): kD4Total = 326 values at the kD4Off* offsets.
// Returns false if the blocks do not have that structure to within `tol`
// relative to their largest entry.
bool interior_d4_blocks(const double* B, double* C, double tol);

// Operand table of the matrix-instruction interior apply (mfma_patch.h):
// A[(blk * 4 + c) * 64 + lane] = entry (row lane % 16, column 4c + lane / 16)
// of block blk of W1, rows and columns ordered by quarter items.  The
// output rows of the 16x16x4 instructions are spread differently over the
// lanes in FP64 (row i in quarter i % 4, element i / 4) and FP32 (quarter
// i / 4, element i % 4); the row order follows `fp64_layout`.
constexpr int kMfmaTable = 4 * 4 * 64;
void mfma_interior_table(const double* B1, bool fp64_layout, double* A);

// Per-level device table of patch operators: the 25 dense weighted inverses
// (51 x 51 each) followed by the 651 reflection-block values of the
// interior one.
constexpr int kDenseTable = kClasses * kSlots * kSlots;
constexpr int kLevelTable = kDenseTable + 651;

}  // namespace vkmg
