// Fine Wilson-clover operator: fields and launchers.
#pragma once
#include "common.h"

namespace mgm {

struct Geom {
  int X, Y, Z, T;
  int64_t V;
  int antiperiodic;
};

struct FineOp {
  Context* ctx = nullptr;
  Geom g{};
  double m0 = 0, csw = 0;
  // links [mu][9][V] complex, clover (+ mass) [72][V] real: two 6x6 Hermitian
  // chirality blocks per site, each 6 diagonal reals then 15 complex lower
  // entries C[i][j] (i > j) in row order.
  double2* U64 = nullptr;
  float2* U32 = nullptr;
  __half2* U16 = nullptr;
  double* C64 = nullptr;
  float* C32 = nullptr;
  __half* C16 = nullptr;

  static void layout(Arena& a, const Geom& g, FineOp* op);
  void build(const double* gauge_host);
  // y = D x, nrhs vectors in dof-major layout of precision p
  void apply(mgm_prec p, const void* x, void* y, int nrhs) const;
  // the same, also writing per-block sums of y^H x and |y|^2 per rhs to
  // dpart[2][nrhs][nb] (finalised by b_finalize_dot_norm); returns nb, the
  // block count of the launch shape that ran (at most nblocks(p, nrhs, true))
  int64_t apply_dot(mgm_prec p, const void* x, void* y, int nrhs, double2* dpart) const;
  // 256-thread blocks of the site-parallel launch, plain (dot = false) or
  // reducing: (V * nrhs / rhs-per-thread + 255) / 256, an upper bound of every
  // launch shape's block count (sizes the partial sums)
  int64_t nblocks(mgm_prec p, int nrhs, bool dot) const;
  // algorithmic bytes of one application (fields once, spinors in and out)
  double bytes(mgm_prec p, int nrhs) const;
  // One fused minimal-residual smoother step with the previous step's
  // length (FP16 storage, plane-marching shapes only): with omega = qr / qq
  // per rhs (0 where qq is 0) and q = D r (not stored), writes
  // r_next = r - omega q, updates x += omega r in place and writes the block
  // partials of q^H r and |q|^2 to dpart; returns their block count.
  bool step_fusable(mgm_prec p, int nrhs) const;
  int64_t apply_step(mgm_prec p, const void* r, void* r_next, void* x, const double2* qr, const double* qq,
                     int nrhs, double2* dpart) const;
  double step_bytes(mgm_prec p, int nrhs) const;
};

}  // namespace mgm
