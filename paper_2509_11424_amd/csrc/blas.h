// Vector kernels over dof-major multi-RHS vectors (element e -> rhs e % nrhs).
#pragma once
#include "common.h"

namespace mgm {

struct Vec {
  void* p = nullptr;
  int64_t nsite = 0;
  int dof = 0;
  int nrhs = 0;
  mgm_prec prec = MGM_PREC_F64;
  // columns stored in groups of `group` right-hand sides, group-major
  // ([nrhs / group][dof][site][group]); 0: the plain (dof, site, rhs) layout.
  // Only the scaled conversions below read or write grouped vectors.
  int group = 0;
  int gs() const { return group > 0 ? group : nrhs; }
  int64_t n() const { return nsite * dof * nrhs; }
  size_t bytes() const { return (size_t)n() * prec_bytes(prec); }
  Vec with(void* q) const {
    Vec v = *this;
    v.p = q;
    return v;
  }
  Vec as(mgm_prec pr, void* q) const {
    Vec v = *this;
    v.prec = pr;
    v.p = q;
    return v;
  }
};

// Reduction scratch: partial sums [blocks][K][nrhs] (complex, FP64).
struct Scratch {
  double2* partial = nullptr;
  size_t cap = 0;  // complex entries
};

constexpr int kRedBlocksMax = 1024;

// ---- elementwise ----
void b_zero(Context* c, Vec x);
void b_copy(Context* c, Vec dst, Vec src);  // converting copy, same shape
// y += sgn * a[r] * x   (a: device complex per rhs; nullptr means 1)
void b_axpy(Context* c, const double2* a, double sgn, Vec x, Vec y);
// y = x + sgn * a[r] * y
void b_xpay(Context* c, Vec x, const double2* a, double sgn, Vec y);
// dst[e] = s[r] * src[e] (converting copy with a per-rhs real scale; either
// side may be grouped)
void b_copy_scaled(Context* c, Vec dst, Vec src, const double* s);
// dst[e] = s[r] * (a[e] - b[e]) (converting, per-rhs real scale; dst may be
// grouped)
void b_sub_scaled(Context* c, Vec dst, Vec a, Vec b, const double* s);
// dst[e] += s[r] * src[e] (converting, per-rhs real scale; src may be
// grouped)
void b_add_scaled(Context* c, Vec dst, Vec src, const double* s);
// s[r] = sqrt(target2 / n2[r]) and inv[r] = 1 / s[r] (both 0 where n2[r] = 0;
// n2 == nullptr stands for n2[r] = 1)
void b_unit_scales(Context* c, const double* n2, double target2, int nrhs, double* s, double* inv);
// x *= s (host real)
void b_scal(Context* c, Vec x, double s);
// x[r] *= 1/sqrt(n2[r]) (0 if n2 == 0); also writes beta[r] = sqrt(n2[r]) if beta != nullptr
void b_normalize(Context* c, Vec x, const double* n2, double* beta);
// x[r] *= m[r] (device real, per rhs)
void b_scale_rhs(Context* c, Vec x, const double* m);
// minimal-residual update: alpha = qr[r] / qq[r]; y += alpha rho; rho -= alpha q
// (rho_in: read the old rho from there instead; y_zero: y = alpha rho, y not read)
void b_mr_update(Context* c, const double2* qr, const double* qq, Vec rho, Vec q, Vec y,
                 const Vec* rho_in = nullptr, bool y_zero = false);

// ---- reductions (out in device memory, FP64) ----
void b_dot(Context* c, Scratch& s, Vec x, Vec y, double2* out);          // out[r] = x^H y
void b_norm2(Context* c, Scratch& s, Vec x, double* out);                 // out[r] = |x|^2
// r = b - r and out[r] = |r|^2 (of the stored values) in one sweep
void b_rsub_norm2(Context* c, Scratch& s, Vec b, Vec r, double* out);
void b_dot_norm(Context* c, Scratch& s, Vec q, Vec rho, double2* qr, double* qq);  // q^H rho, |q|^2
// sums per-block partials [2][nrhs][nblk] (q^H rho, then |q|^2) written by a fused kernel
void b_finalize_dot_norm(Context* c, Scratch& s, const double2* part, int64_t nblk, int nrhs, double2* qr,
                         double* qq);
// out[i*nrhs + r] = V_i^H w for i < k; basis V_i = base + i * stride (elements)
void b_multidot(Context* c, Scratch& s, Vec base, int64_t stride, int k, Vec w, double2* out);
// w += sgn * sum_i h[i*nrhs + r] V_i (overwrite: w = sgn * sum ..., w not read);
// if n2 != nullptr also n2[r] = |w|^2 after the update
void b_multiaxpy(Context* c, Scratch& s, Vec base, int64_t stride, int k, const double2* h, double sgn,
                 Vec w, double* n2, bool overwrite = false);
// w -= sum_i h_i V_i and out[i*nrhs + r] = V_i^H w (updated), one sweep, k <= kFusedGS
constexpr int kFusedGS = 16;
void b_multiaxpy_dot(Context* c, Scratch& s, Vec base, int64_t stride, int k, const double2* h, Vec w,
                     double2* out);

// ---- small dense kernels for (F)GMRES, one thread per rhs ----
struct Givens {
  double2* R = nullptr;    // [m][m][nrhs] upper triangle (column-major by j)
  double* cs = nullptr;    // [m][nrhs]
  double2* sn = nullptr;   // [m][nrhs]
  double2* g = nullptr;    // [m+1][nrhs]
  double2* h = nullptr;    // [m+1][nrhs] scratch column (first pass)
  double2* h2 = nullptr;   // [m+1][nrhs] scratch column (second pass)
  double* beta = nullptr;  // [nrhs] subdiagonal norm
  double* est = nullptr;   // [nrhs] |g_{j+1}| residual estimate
  double2* y = nullptr;    // [m][nrhs]
  int m = 0;
};
// g = (beta0, 0, ...); beta0 given as |r|^2 per rhs
void k_gmres_start(Context* c, Givens& G, const double* r2, int nrhs);
// column j: combine h + h2, apply old rotations, new rotation with beta (|w|^2 given)
// (reorth: the column is h + h2, the projections of both Gram-Schmidt passes; else h)
void k_gmres_column(Context* c, Givens& G, int j, const double* w2, int nrhs, bool reorth = true);
// back substitution R y = g for k columns
void k_gmres_solve(Context* c, Givens& G, int k, int nrhs);

}  // namespace mgm
