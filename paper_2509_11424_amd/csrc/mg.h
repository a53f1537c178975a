// Aggregation transfers, block orthonormalisation and coarse stencils.
#pragma once
#include "blas.h"
#include "fine.h"

namespace mgm {

// Lattice of one level: sites and dof per site (dof = 2 * half, chirality
// chi owns dof chi*half .. chi*half + half - 1).
struct LGeom {
  int dims[4];
  int64_t V;
  int dof;
};

// P_l between level l (fine side) and level l+1: aggregates are blocks of
// b[mu] sites; P is stored per (aggregate, chirality) as [a][chi][row][k]
// with row = loc*half + j (loc: lexicographic site inside the aggregate).
struct TGeom {
  LGeom f, c;
  int b[4];
  int ntv, bvol, half, rows;
};

struct Transfer {
  Context* ctx = nullptr;
  TGeom t{};
  double2* P64 = nullptr;
  __half2* P16 = nullptr;  // FP16 copy used by the mixed-precision V-cycle
  // restrict: y_c = P^H x ; prolong: mode 0 y = P x_c, 1 y = x - P x_c, 2 y += P x_c
  void restrict_(mgm_prec p, const void* x, void* yc, int nrhs) const;
  void prolong(mgm_prec p, const void* xc, const void* x, void* y, int nrhs, int mode) const;
  // FP32 transfers whose fine input is FP16 scaled per rhs by xs:
  // y_c = P^H (xs x16) and y = xs x16 + P x_c
  // x16 in column groups of xgs right-hand sides (0: plain layout)
  void restrict16(const __half2* x16, const double* xs, float2* yc, int nrhs, int xgs = 0) const;
  void prolong16(const float2* xc, const __half2* x16, const double* xs, float2* y, int nrhs, int xgs = 0) const;
  double bytes(mgm_prec p, int nrhs) const;
};

// Nine-point coarse stencil, stored [dir][i][j][site] (site fastest) so a
// wave of consecutive sites reads consecutive addresses.
struct CoarseOp {
  Context* ctx = nullptr;
  LGeom g{};
  int d = 0;
  double2* A64 = nullptr;
  float2* A32 = nullptr;
  double2* Ap64 = nullptr;  // FP64 MFMA operand layout (see coarse_mfma.hip)
  void* Abf = nullptr;      // BF16 MFMA operand layout
  void apply(mgm_prec p, const void* x, void* y, int nrhs) const;
  double bytes(mgm_prec p, int nrhs) const;
};

TGeom make_tgeom(const LGeom& f, const int b[4], int ntv);
LGeom coarse_geom(const LGeom& f, const int b[4], int ntv);

// int64 [Vc][2][rows] map: flat fine dof index of each block row
void mg_agg_map(Context* c, const TGeom& t, int64_t* out_dev);
// Orthonormalise test vectors tv (dof-major FP64, ntv right-hand sides) into
// P (FP64, [a][chi][row][k]); rank_flag (device int) set to 1 on breakdown.
void mg_block_mgs2(Context* c, const TGeom& t, const double2* tv, double2* P, int* rank_flag);
// Galerkin products D_c = P^H D P into the stencil layout of CoarseOp
void mg_galerkin_fine(Context* c, const FineOp& op, const Transfer& T, CoarseOp& out);
void mg_galerkin_coarse(Context* c, const CoarseOp& op, const Transfer& T, CoarseOp& out);
// precision copies
void mg_convert_P(Context* c, Transfer& T);
void mg_convert_A(Context* c, CoarseOp& A);
void mg_mfma_pack(Context* c, CoarseOp& A);
size_t mg_mfma_bytes(const CoarseOp& A);
void coarse_apply_mfma(const CoarseOp& A, const float2* x, float2* y, int nrhs);
void mg_mfma64_pack(Context* c, CoarseOp& A);
size_t mg_mfma64_bytes(const CoarseOp& A);
void coarse_apply_mfma64(const CoarseOp& A, const double2* x, double2* y, int nrhs);
// FP32 copy in the same packed operand layout (made from the FP64 pack)
void mg_mfma32_pack(Context* c, CoarseOp& A);
size_t mg_mfma32_bytes(const CoarseOp& A);
void coarse_apply_mfma32(const CoarseOp& A, const float2* x, float2* y, int nrhs);

}  // namespace mgm
