// Blocks of k vectors of one level stored as one dof-major batch: element
// (dof, site, column) at (dof * V + site) * k + column, i.e. a row-major
// rows x k matrix with rows = dof * V + site.  Tall-skinny products and the
// orthonormalisation of such blocks (inexact deflation, test-vector
// refinement).
#pragma once
#include <complex>
#include <vector>

#include "common.h"

namespace mgm {

// Partial-sum entries a product C = A^H B with ka, kb <= k_max needs.
size_t blk_part_entries(int ka_max, int kb_max);
// C (device, ka x kb, row-major) = A^H B over `rows` rows (deterministic).
void blk_ahb(Context* c, const double2* A, int ka, const double2* B, int kb, int64_t rows, double2* part,
             size_t part_cap, double2* C);
// W <- W M in place (M: k x k device, row-major).
void blk_rowmul(Context* c, double2* W, int k, int64_t rows, const double2* M);
// out[row][j] = sign(row) W[row][c0 + j] for j < b (sign -1 on dof >= dof/2
// when g5: Gamma5 of the level, chirality 1), out a batch of b columns.
void blk_gather(Context* c, const double2* W, int k, int c0, int b, int64_t nsite, int dof, bool g5, double2* out);
void blk_scatter(Context* c, const double2* in, int k, int c0, int b, int64_t rows, double2* W);
// V <- V R^-1 with V^H V = R^H R (R upper triangular, positive diagonal):
// one CholeskyQR pass (the caller applies it twice).  C and M hold k x k
// entries.  RANK_DEFICIENT when a column's component outside the earlier ones
// falls below 1e-12 of its norm.
void blk_cholqr(Context* c, double2* V, int k, int64_t rows, double2* part, size_t part_cap, double2* C, double2* M);
// Host copy of a device k x kb block of complex values.
std::vector<std::complex<double>> blk_fetch(Context* c, const double2* C, size_t n);

}  // namespace mgm
