// BLAS-1 kernels over dof-major multi-RHS vectors and the small dense
// kernels of device-resident (F)GMRES.  Reductions accumulate in FP64 and are
// deterministic: fixed per-thread element sets, a fixed-order LDS tree per
// block and a fixed-order sum over block partials in a second kernel.
#include "blas.h"
#include "group.h"

namespace mgm {

#define DISPATCH_PREC(pr, TAG, ...)                                     \
  switch (pr) {                                                         \
    case MGM_PREC_F64: { using TAG = F64; __VA_ARGS__; } break;         \
    case MGM_PREC_F32: { using TAG = F32; __VA_ARGS__; } break;         \
    case MGM_PREC_F16: { using TAG = F16; __VA_ARGS__; } break;         \
    default: throw Error(MGM_ERR_INVALID_ARG, "unsupported vector precision"); \
  }

template <class P>
__device__ __forceinline__ cx<double> ldd(const void* p, int64_t i) {
  cx<typename P::R> v = P::ld((const typename P::S*)p, i);
  return {(double)v.re, (double)v.im};
}
template <class P>
__device__ __forceinline__ void std_(void* p, int64_t i, cx<double> v) {
  P::st((typename P::S*)p, i, cx<typename P::R>{(typename P::R)v.re, (typename P::R)v.im});
}

// rhs index of a grid-stride loop, advanced without 64-bit division
struct RhsIter {
  int r, step, nrhs;
  __device__ RhsIter(int64_t i0, int64_t stride, int nr)
      : r((int)(i0 % nr)), step((int)(stride % nr)), nrhs(nr) {}
  __device__ void next() {
    r += step;
    if (r >= nrhs) r -= nrhs;
  }
};

// (row, rhs) of element i of a plain (row, rhs) block, advanced by a
// fixed stride
struct RowRhsIter {
  int64_t row, step_row;
  int r, step_r, nrhs;
  __device__ RowRhsIter(int64_t i0, int64_t stride, int nr)
      : row(i0 / nr), step_row(stride / nr), r((int)(i0 % nr)), step_r((int)(stride % nr)), nrhs(nr) {}
  __device__ void next() {
    row += step_row;
    r += step_r;
    if (r >= nrhs) {
      r -= nrhs;
      row++;
    }
  }
};

// Routines that apply per-rhs factors or reduce per rhs read the plain
// (dof, site, rhs) layout only; a vector with column groups reaching them is
// a caller's mistake.
static void plain_layout(const Vec& v) {
  MGM_CHECK(v.group == 0, MGM_ERR_INVALID_ARG, "vector with column groups passed to a plain-layout routine");
}

static inline unsigned ew_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 65536 * 4 ? b : 65536 * 4);
}

// ------------------------------------------------------------ elementwise

__global__ void k_zero_bytes(uint4* p, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0, 0, 0, 0);
}

void b_zero(Context* c, Vec x) {
  size_t b = x.bytes();
  if (b == 0) return;
  // all vectors are carved with 256-byte granularity, so rounding up is safe
  int64_t n16 = (int64_t)((b + 15) / 16);
  hipLaunchKernelGGL(k_zero_bytes, dim3(ew_blocks(n16)), dim3(256), 0, c->stream, (uint4*)x.p, n16);
  MGM_LAUNCH_CHECK();
}

template <class Pd, class Ps>
__global__ void k_copy(void* d, const void* s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    std_<Pd>(d, i, ldd<Ps>(s, i));
}

void b_copy(Context* c, Vec dst, Vec src) {
  int64_t n = src.n();
  MGM_CHECK(dst.n() == n, MGM_ERR_INVALID_ARG, "copy: shape mismatch");
  if (n == 0) return;
  DISPATCH_PREC(dst.prec, PD, DISPATCH_PREC(src.prec, PS,
      hipLaunchKernelGGL((k_copy<PD, PS>), dim3(ew_blocks(n)), dim3(256), 0, c->stream, dst.p, src.p, n)));
  MGM_LAUNCH_CHECK();
}

// The scaled conversions take the column-group size of each operand (gd for
// the destination, gs for the source; nrhs for a plain operand).
template <class PD, class PS>
__global__ void k_copy_scaled(void* dst, const void* src, int64_t n, int nrhs, const double* s, int gd, int gs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gd == nrhs && gs == nrhs) {
    for (RhsIter it(i, stride, nrhs); i < n; i += stride, it.next()) std_<PD>(dst, i, s[it.r] * ldd<PS>(src, i));
    return;
  }
  const int64_t rows = n / nrhs;
  for (RowRhsIter it(i, stride, nrhs); i < n; i += stride, it.next())
    std_<PD>(dst, grouped_index(it.row, it.r, nrhs, gd, rows),
             s[it.r] * ldd<PS>(src, grouped_index(it.row, it.r, nrhs, gs, rows)));
}
static void check_groups(const Vec& v) {
  MGM_CHECK(v.group == 0 || (v.group > 0 && v.nrhs % v.group == 0), MGM_ERR_INVALID_ARG,
            "column groups must divide the rhs count");
}
void b_copy_scaled(Context* c, Vec dst, Vec src, const double* s) {
  int64_t n = src.n();
  MGM_CHECK(dst.n() == n && dst.nrhs == src.nrhs, MGM_ERR_INVALID_ARG, "copy: shape mismatch");
  check_groups(dst);
  check_groups(src);
  if (n == 0) return;
  DISPATCH_PREC(dst.prec, PD, DISPATCH_PREC(src.prec, PS,
      hipLaunchKernelGGL((k_copy_scaled<PD, PS>), dim3(ew_blocks(n)), dim3(256), 0, c->stream, dst.p, src.p, n,
                         src.nrhs, s, dst.gs(), src.gs())));
  MGM_LAUNCH_CHECK();
}

template <class PD, class PS>
__global__ void k_sub_scaled(void* dst, const void* a, const void* b, int64_t n, int nrhs, const double* s, int gd) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gd == nrhs) {
    for (RhsIter it(i, stride, nrhs); i < n; i += stride, it.next())
      std_<PD>(dst, i, s[it.r] * (ldd<PS>(a, i) - ldd<PS>(b, i)));
    return;
  }
  const int64_t rows = n / nrhs;
  for (RowRhsIter it(i, stride, nrhs); i < n; i += stride, it.next())
    std_<PD>(dst, grouped_index(it.row, it.r, nrhs, gd, rows), s[it.r] * (ldd<PS>(a, i) - ldd<PS>(b, i)));
}
void b_sub_scaled(Context* c, Vec dst, Vec a, Vec b, const double* s) {
  int64_t n = a.n();
  MGM_CHECK(dst.n() == n && b.n() == n && dst.nrhs == a.nrhs && b.prec == a.prec, MGM_ERR_INVALID_ARG,
            "sub: shape mismatch");
  MGM_CHECK(a.group == 0 && b.group == 0, MGM_ERR_INVALID_ARG, "sub: grouped operands");
  check_groups(dst);
  if (n == 0) return;
  DISPATCH_PREC(dst.prec, PD, DISPATCH_PREC(a.prec, PS,
      hipLaunchKernelGGL((k_sub_scaled<PD, PS>), dim3(ew_blocks(n)), dim3(256), 0, c->stream, dst.p, a.p, b.p,
                         n, a.nrhs, s, dst.gs())));
  MGM_LAUNCH_CHECK();
}

template <class PD, class PS>
__global__ void k_add_scaled(void* dst, const void* src, int64_t n, int nrhs, const double* s, int gs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gs == nrhs) {
    for (RhsIter it(i, stride, nrhs); i < n; i += stride, it.next())
      std_<PD>(dst, i, ldd<PD>(dst, i) + s[it.r] * ldd<PS>(src, i));
    return;
  }
  const int64_t rows = n / nrhs;
  for (RowRhsIter it(i, stride, nrhs); i < n; i += stride, it.next())
    std_<PD>(dst, i, ldd<PD>(dst, i) + s[it.r] * ldd<PS>(src, grouped_index(it.row, it.r, nrhs, gs, rows)));
}
void b_add_scaled(Context* c, Vec dst, Vec src, const double* s) {
  int64_t n = src.n();
  MGM_CHECK(dst.n() == n && dst.nrhs == src.nrhs, MGM_ERR_INVALID_ARG, "add: shape mismatch");
  MGM_CHECK(dst.group == 0, MGM_ERR_INVALID_ARG, "add: grouped destination");
  check_groups(src);
  if (n == 0) return;
  DISPATCH_PREC(dst.prec, PD, DISPATCH_PREC(src.prec, PS,
      hipLaunchKernelGGL((k_add_scaled<PD, PS>), dim3(ew_blocks(n)), dim3(256), 0, c->stream, dst.p, src.p, n,
                         src.nrhs, s, src.gs())));
  MGM_LAUNCH_CHECK();
}

__global__ void k_unit_scales(const double* n2, double target2, int nrhs, double* s, double* inv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const double d = n2 ? n2[r] : 1.0;  // no norms given: unit columns
  const double f = d > 0.0 ? sqrt(target2 / d) : 0.0;
  s[r] = f;
  inv[r] = f > 0.0 ? 1.0 / f : 0.0;
}
void b_unit_scales(Context* c, const double* n2, double target2, int nrhs, double* s, double* inv) {
  hipLaunchKernelGGL(k_unit_scales, dim3(nblocks_for(nrhs, 64)), dim3(64), 0, c->stream, n2, target2, nrhs, s, inv);
  MGM_LAUNCH_CHECK();
}

template <class P>
__global__ void k_axpy(const double2* a, double sgn, const void* x, void* y, int64_t n, int nrhs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (RhsIter it(i, stride, nrhs); i < n; i += stride, it.next()) {
    const int r = it.r;
    cx<double> al = a ? cx<double>{a[r].x, a[r].y} : cx<double>{1.0, 0.0};
    al = sgn * al;
    cx<double> yv = ldd<P>(y, i);
    fma_(yv, al, ldd<P>(x, i));
    std_<P>(y, i, yv);
  }
}
void b_axpy(Context* c, const double2* a, double sgn, Vec x, Vec y) {
  plain_layout(x);
  plain_layout(y);
  int64_t n = x.n();
  MGM_CHECK(y.n() == n && x.prec == y.prec, MGM_ERR_INVALID_ARG, "axpy: mismatch");
  if (n == 0) return;
  DISPATCH_PREC(x.prec, P, hipLaunchKernelGGL(k_axpy<P>, dim3(ew_blocks(n)), dim3(256), 0, c->stream,
                                              a, sgn, x.p, y.p, n, x.nrhs));
  MGM_LAUNCH_CHECK();
}

template <class P>
__global__ void k_xpay(const void* x, const double2* a, double sgn, void* y, int64_t n, int nrhs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (RhsIter it(i, stride, nrhs); i < n; i += stride, it.next()) {
    const int r = it.r;
    cx<double> al = a ? cx<double>{a[r].x, a[r].y} : cx<double>{1.0, 0.0};
    al = sgn * al;
    cx<double> v = ldd<P>(x, i);
    fma_(v, al, ldd<P>(y, i));
    std_<P>(y, i, v);
  }
}
void b_xpay(Context* c, Vec x, const double2* a, double sgn, Vec y) {
  plain_layout(x);
  plain_layout(y);
  int64_t n = x.n();
  MGM_CHECK(y.n() == n && x.prec == y.prec, MGM_ERR_INVALID_ARG, "xpay: mismatch");
  if (n == 0) return;
  DISPATCH_PREC(x.prec, P, hipLaunchKernelGGL(k_xpay<P>, dim3(ew_blocks(n)), dim3(256), 0, c->stream,
                                              x.p, a, sgn, y.p, n, x.nrhs));
  MGM_LAUNCH_CHECK();
}

template <class P>
__global__ void k_scal(void* x, double s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    std_<P>(x, i, s * ldd<P>(x, i));
}
void b_scal(Context* c, Vec x, double s) {
  int64_t n = x.n();
  if (n == 0) return;
  DISPATCH_PREC(x.prec, P, hipLaunchKernelGGL(k_scal<P>, dim3(ew_blocks(n)), dim3(256), 0, c->stream, x.p, s, n));
  MGM_LAUNCH_CHECK();
}

template <class P>
__global__ void k_normalize(void* x, const double* n2, double* beta, int64_t n, int nrhs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (RhsIter it(i, stride, nrhs); i < n; i += stride, it.next()) {
    const int r = it.r;
    double b = sqrt(n2[r]);
    double s = b > 0.0 ? 1.0 / b : 0.0;
    std_<P>(x, i, s * ldd<P>(x, i));
    if (beta && i < nrhs) beta[r] = b;
  }
}
void b_normalize(Context* c, Vec x, const double* n2, double* beta) {
  plain_layout(x);
  int64_t n = x.n();
  if (n == 0) return;
  DISPATCH_PREC(x.prec, P, hipLaunchKernelGGL(k_normalize<P>, dim3(ew_blocks(n)), dim3(256), 0, c->stream,
                                              x.p, n2, beta, n, x.nrhs));
  MGM_LAUNCH_CHECK();
}

template <class P>
__global__ void k_scale_rhs(void* x, const double* m, int64_t n, int nrhs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (RhsIter it(i, stride, nrhs); i < n; i += stride, it.next()) std_<P>(x, i, m[it.r] * ldd<P>(x, i));
}
void b_scale_rhs(Context* c, Vec x, const double* m) {
  plain_layout(x);
  int64_t n = x.n();
  if (n == 0) return;
  DISPATCH_PREC(x.prec, P, hipLaunchKernelGGL(k_scale_rhs<P>, dim3(ew_blocks(n)), dim3(256), 0, c->stream,
                                              x.p, m, n, x.nrhs));
  MGM_LAUNCH_CHECK();
}

template <class P>
__global__ __launch_bounds__(256) void k_mr_update(const double2* qr, const double* qq, const void* rho_in,
                                                   void* rho, const void* q, void* y, int64_t n, int nrhs,
                                                   int y_zero) {
  __shared__ double2 sa[256];  // alpha = qr / qq per rhs (nrhs <= 256)
  for (int r = threadIdx.x; r < nrhs; r += blockDim.x) {
    const double d = qq[r];
    sa[r] = d > 0.0 ? make_double2(qr[r].x / d, qr[r].y / d) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (RhsIter it(i, stride, nrhs); i < n; i += stride, it.next()) {
    const cx<double> al = {sa[it.r].x, sa[it.r].y};
    cx<double> rv = ldd<P>(rho_in, i);
    cx<double> yv = y_zero ? cx<double>{0, 0} : ldd<P>(y, i);
    fma_(yv, al, rv);
    cx<double> qv = ldd<P>(q, i);
    rv = rv - al * qv;
    std_<P>(y, i, yv);
    std_<P>(rho, i, rv);
  }
}
void b_mr_update(Context* c, const double2* qr, const double* qq, Vec rho, Vec q, Vec y, const Vec* rho_in,
                 bool y_zero) {
  plain_layout(rho);
  plain_layout(q);
  plain_layout(y);
  if (rho_in) plain_layout(*rho_in);
  int64_t n = rho.n();
  if (n == 0) return;
  MGM_CHECK(rho.nrhs >= 1 && rho.nrhs <= 256, MGM_ERR_INVALID_ARG, "at most 256 right-hand sides");
  MGM_CHECK(rho_in == nullptr || (rho_in->n() == n && rho_in->prec == rho.prec), MGM_ERR_INVALID_ARG,
            "mr update: shape mismatch");
  const void* src = rho_in ? rho_in->p : rho.p;
  DISPATCH_PREC(rho.prec, P, hipLaunchKernelGGL(k_mr_update<P>, dim3(ew_blocks(n)), dim3(256), 0, c->stream,
                                                qr, qq, src, rho.p, q.p, y.p, n, rho.nrhs, y_zero ? 1 : 0));
  MGM_LAUNCH_CHECK();
}

// ------------------------------------------------------------- reductions

struct RedPlan {
  unsigned blocks;
  int64_t J;   // threads per rhs
  int64_t m;   // elements per rhs (n / nrhs)
};
static RedPlan red_plan(int64_t n, int nrhs) {
  RedPlan p;
  int64_t want = (n + 255) / 256;
  if (want > kRedBlocksMax) want = kRedBlocksMax;
  if (want < 1) want = 1;
  // at least one full set of rhs lanes
  while (want * 256 < nrhs) want++;
  p.blocks = (unsigned)want;
  p.J = (int64_t)want * 256 / nrhs;
  p.m = n / nrhs;
  return p;
}

// Block reduction of K complex values per thread into partial[blk][K][nrhs].
template <int K>
__device__ __forceinline__ void block_store(double2 (&v)[K], double2* partial, int nrhs) {
  __shared__ double2 sh[256];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * blockDim.x;
#pragma unroll
  for (int k = 0; k < K; k++) {
    sh[t] = v[k];
    __syncthreads();
    if (t < nrhs) {
      int t0 = (int)(((t - base % nrhs) % nrhs + nrhs) % nrhs);
      double sr = 0, si = 0;
      for (int u = t0; u < (int)blockDim.x; u += nrhs) {
        sr += sh[u].x;
        si += sh[u].y;
      }
      partial[((int64_t)blockIdx.x * K + k) * nrhs + t] = make_double2(sr, si);
    }
    __syncthreads();
  }
}

// Second stage of every reduction: one 64-lane wave per output entry; lane j
// sums block partials j, j+64, ... and a fixed shuffle tree adds the lanes.
__device__ __forceinline__ double2 wave_sum_partials(const double2* partial, int nblk, int stride, int i) {
  double a = 0, b = 0;
  for (int k = threadIdx.x; k < nblk; k += 64) {
    double2 v = partial[(int64_t)k * stride + i];
    a += v.x;
    b += v.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  return make_double2(a, b);
}

// out[out_off + i] = sum_b partial[b][K][nrhs] entry i, for i < cnt (grid = cnt)
__global__ void k_finalize_c(const double2* partial, int nblk, int K, int nrhs, int cnt, double2* out,
                             int64_t out_off) {
  const int i = blockIdx.x;
  double2 v = wave_sum_partials(partial, nblk, K * nrhs, i);
  if (threadIdx.x == 0) out[out_off + i] = v;
}
// real parts, i < K * nrhs (grid = K * nrhs)
__global__ void k_finalize_r(const double2* partial, int nblk, int K, int nrhs, double* out) {
  const int i = blockIdx.x;
  double2 v = wave_sum_partials(partial, nblk, K * nrhs, i);
  if (threadIdx.x == 0) out[i] = v.x;
}
// q^H rho (slot 0) and |q|^2 (slot 1) -> separate outputs (grid = 2 * nrhs)
__global__ void k_finalize_dn(const double2* partial, int nblk, int nrhs, double2* qr, double* qq) {
  const int i = blockIdx.x;
  double2 v = wave_sum_partials(partial, nblk, 2 * nrhs, i);
  if (threadIdx.x == 0) {
    if (i < nrhs)
      qr[i] = v;
    else
      qq[i - nrhs] = v.x;
  }
}

static void need(Scratch& s, size_t entries) {
  MGM_CHECK(s.partial != nullptr && entries <= s.cap, MGM_ERR_WORKSPACE, "reduction scratch too small");
}

template <class P>
__global__ void k_dot(const void* x, const void* y, int nrhs, RedPlan pl, double2* partial) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 v[1] = {make_double2(0, 0)};
  if (g < pl.J * nrhs) {
    int r = (int)(g % nrhs);
    int64_t j = g / nrhs;
    cx<double> a = {0, 0};
    for (int64_t m = j; m < pl.m; m += pl.J) {
      int64_t e = m * nrhs + r;
      fmac_(a, ldd<P>(x, e), ldd<P>(y, e));
    }
    v[0] = make_double2(a.re, a.im);
  }
  block_store<1>(v, partial, nrhs);
}
void b_dot(Context* c, Scratch& s, Vec x, Vec y, double2* out) {
  plain_layout(x);
  plain_layout(y);
  RedPlan pl = red_plan(x.n(), x.nrhs);
  need(s, (size_t)pl.blocks * x.nrhs);
  DISPATCH_PREC(x.prec, P, hipLaunchKernelGGL(k_dot<P>, dim3(pl.blocks), dim3(256), 0, c->stream, x.p, y.p,
                                              x.nrhs, pl, s.partial));
  hipLaunchKernelGGL(k_finalize_c, dim3(x.nrhs), dim3(64), 0, c->stream, s.partial,
                     (int)pl.blocks, 1, x.nrhs, x.nrhs, out, (int64_t)0);
  MGM_LAUNCH_CHECK();
}

template <class P>
__global__ void k_norm2(const void* x, int nrhs, RedPlan pl, double2* partial) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 v[1] = {make_double2(0, 0)};
  if (g < pl.J * nrhs) {
    int r = (int)(g % nrhs);
    int64_t j = g / nrhs;
    double a = 0;
    for (int64_t m = j; m < pl.m; m += pl.J) a += norm2(ldd<P>(x, m * nrhs + r));
    v[0] = make_double2(a, 0);
  }
  block_store<1>(v, partial, nrhs);
}
void b_norm2(Context* c, Scratch& s, Vec x, double* out) {
  plain_layout(x);
  RedPlan pl = red_plan(x.n(), x.nrhs);
  need(s, (size_t)pl.blocks * x.nrhs);
  DISPATCH_PREC(x.prec, P, hipLaunchKernelGGL(k_norm2<P>, dim3(pl.blocks), dim3(256), 0, c->stream, x.p,
                                              x.nrhs, pl, s.partial));
  hipLaunchKernelGGL(k_finalize_r, dim3(x.nrhs), dim3(64), 0, c->stream, s.partial,
                     (int)pl.blocks, 1, x.nrhs, out);
  MGM_LAUNCH_CHECK();
}

// r = b - r with the norms of the stored r
template <class P>
__global__ void k_rsub_norm2(const void* b, void* r, int nrhs, RedPlan pl, double2* partial) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 v[1] = {make_double2(0, 0)};
  if (g < pl.J * nrhs) {
    int rr = (int)(g % nrhs);
    int64_t j = g / nrhs;
    double a = 0;
    for (int64_t m = j; m < pl.m; m += pl.J) {
      const int64_t e = m * nrhs + rr;
      std_<P>(r, e, ldd<P>(b, e) - ldd<P>(r, e));
      a += norm2(ldd<P>(r, e));
    }
    v[0] = make_double2(a, 0);
  }
  block_store<1>(v, partial, nrhs);
}
void b_rsub_norm2(Context* c, Scratch& s, Vec b, Vec r, double* out) {
  plain_layout(b);
  plain_layout(r);
  MGM_CHECK(b.n() == r.n() && b.nrhs == r.nrhs && b.prec == r.prec, MGM_ERR_INVALID_ARG, "rsub: shape mismatch");
  RedPlan pl = red_plan(r.n(), r.nrhs);
  need(s, (size_t)pl.blocks * r.nrhs);
  DISPATCH_PREC(r.prec, P, hipLaunchKernelGGL(k_rsub_norm2<P>, dim3(pl.blocks), dim3(256), 0, c->stream, b.p,
                                              r.p, r.nrhs, pl, s.partial));
  hipLaunchKernelGGL(k_finalize_r, dim3(r.nrhs), dim3(64), 0, c->stream, s.partial,
                     (int)pl.blocks, 1, r.nrhs, out);
  MGM_LAUNCH_CHECK();
}

template <class P>
__global__ void k_dot_norm(const void* q, const void* rho, int nrhs, RedPlan pl, double2* partial) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 v[2] = {make_double2(0, 0), make_double2(0, 0)};
  if (g < pl.J * nrhs) {
    int r = (int)(g % nrhs);
    int64_t j = g / nrhs;
    cx<double> a = {0, 0};
    double d = 0;
    for (int64_t m = j; m < pl.m; m += pl.J) {
      int64_t e = m * nrhs + r;
      cx<double> qv = ldd<P>(q, e);
      fmac_(a, qv, ldd<P>(rho, e));
      d += norm2(qv);
    }
    v[0] = make_double2(a.re, a.im);
    v[1] = make_double2(d, 0);
  }
  block_store<2>(v, partial, nrhs);
}
void b_dot_norm(Context* c, Scratch& s, Vec q, Vec rho, double2* qr, double* qq) {
  plain_layout(q);
  plain_layout(rho);
  RedPlan pl = red_plan(q.n(), q.nrhs);
  need(s, (size_t)pl.blocks * 2 * q.nrhs);
  DISPATCH_PREC(q.prec, P, hipLaunchKernelGGL(k_dot_norm<P>, dim3(pl.blocks), dim3(256), 0, c->stream, q.p,
                                              rho.p, q.nrhs, pl, s.partial));
  hipLaunchKernelGGL(k_finalize_dn, dim3(2 * q.nrhs), dim3(64), 0, c->stream, s.partial,
                     (int)pl.blocks, q.nrhs, qr, qq);
  MGM_LAUNCH_CHECK();
}

template <class P, int KB>
__global__ __launch_bounds__(256) void k_multidot(const void* base, int64_t stride, int k, const void* w, int nrhs,
                                                  RedPlan pl, double2* partial) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 v[KB];
#pragma unroll
  for (int i = 0; i < KB; i++) v[i] = make_double2(0, 0);
  if (g < pl.J * nrhs) {
    int r = (int)(g % nrhs);
    int64_t j = g / nrhs;
    cx<double> a[KB];
#pragma unroll
    for (int i = 0; i < KB; i++) a[i] = {0, 0};
    const typename P::S* B = (const typename P::S*)base;
    for (int64_t m = j; m < pl.m; m += pl.J) {
      int64_t e = m * nrhs + r;
      cx<double> wv = ldd<P>(w, e);
#pragma unroll
      for (int i = 0; i < KB; i++)
        if (i < k) fmac_(a[i], ldd<P>(B + i * stride, e), wv);
    }
#pragma unroll
    for (int i = 0; i < KB; i++) v[i] = make_double2(a[i].re, a[i].im);
  }
  block_store<KB>(v, partial, nrhs);
}
template <class P>
static void launch_multidot(Context* c, const typename P::S* b0, int64_t stride, int kk, Vec w, RedPlan pl,
                            double2* partial) {
  const dim3 nb(pl.blocks), tb(256);
  switch (kk) {
    case 1: hipLaunchKernelGGL((k_multidot<P, 1>), nb, tb, 0, c->stream, b0, stride, kk, w.p, w.nrhs, pl, partial); break;
    case 2: hipLaunchKernelGGL((k_multidot<P, 2>), nb, tb, 0, c->stream, b0, stride, kk, w.p, w.nrhs, pl, partial); break;
    case 3: hipLaunchKernelGGL((k_multidot<P, 3>), nb, tb, 0, c->stream, b0, stride, kk, w.p, w.nrhs, pl, partial); break;
    case 4: hipLaunchKernelGGL((k_multidot<P, 4>), nb, tb, 0, c->stream, b0, stride, kk, w.p, w.nrhs, pl, partial); break;
    case 5: hipLaunchKernelGGL((k_multidot<P, 5>), nb, tb, 0, c->stream, b0, stride, kk, w.p, w.nrhs, pl, partial); break;
    case 6: hipLaunchKernelGGL((k_multidot<P, 6>), nb, tb, 0, c->stream, b0, stride, kk, w.p, w.nrhs, pl, partial); break;
    case 7: hipLaunchKernelGGL((k_multidot<P, 7>), nb, tb, 0, c->stream, b0, stride, kk, w.p, w.nrhs, pl, partial); break;
    default: hipLaunchKernelGGL((k_multidot<P, 8>), nb, tb, 0, c->stream, b0, stride, kk, w.p, w.nrhs, pl, partial); break;
  }
}

void b_multidot(Context* c, Scratch& s, Vec base, int64_t stride, int k, Vec w, double2* out) {
  plain_layout(base);
  plain_layout(w);
  RedPlan pl = red_plan(w.n(), w.nrhs);
  const int KB = 8;
  need(s, (size_t)pl.blocks * KB * w.nrhs);
  for (int i0 = 0; i0 < k; i0 += KB) {
    const int kk = k - i0 < KB ? k - i0 : KB;
    // the chunk's exact size as a template parameter: registers and
    // block-reduction rounds follow the vectors in use
    DISPATCH_PREC(w.prec, P, launch_multidot<P>(c, (const typename P::S*)base.p + i0 * stride, stride, kk, w, pl,
                                                 s.partial));
    hipLaunchKernelGGL(k_finalize_c, dim3(kk * w.nrhs), dim3(64), 0, c->stream, s.partial,
                       (int)pl.blocks, kk, w.nrhs, kk * w.nrhs, out, (int64_t)i0 * w.nrhs);
    MGM_LAUNCH_CHECK();
  }
}

template <class P>
__global__ void k_multiaxpy(const void* base, int64_t stride, int k, const double2* h, double sgn, void* w,
                            int nrhs, RedPlan pl, double2* partial, int want_norm, int overwrite) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 v[1] = {make_double2(0, 0)};
  if (g < pl.J * nrhs) {
    int r = (int)(g % nrhs);
    int64_t j = g / nrhs;
    const typename P::S* B = (const typename P::S*)base;
    double nn = 0;
    for (int64_t m = j; m < pl.m; m += pl.J) {
      int64_t e = m * nrhs + r;
      cx<double> wv = overwrite ? cx<double>{0, 0} : ldd<P>(w, e);
      for (int i = 0; i < k; i++) {
        double2 hh = h[(int64_t)i * nrhs + r];
        cx<double> hc = {sgn * hh.x, sgn * hh.y};
        fma_(wv, hc, ldd<P>(B + i * stride, e));
      }
      std_<P>(w, e, wv);
      if (want_norm) {
        cx<double> st = ldd<P>(w, e);  // norm of the stored (rounded) value
        nn += norm2(st);
      }
    }
    v[0] = make_double2(nn, 0);
  }
  if (want_norm) block_store<1>(v, partial, nrhs);
}
void b_multiaxpy(Context* c, Scratch& s, Vec base, int64_t stride, int k, const double2* h, double sgn, Vec w,
                 double* n2, bool overwrite) {
  plain_layout(base);
  plain_layout(w);
  RedPlan pl = red_plan(w.n(), w.nrhs);
  need(s, (size_t)pl.blocks * w.nrhs);
  DISPATCH_PREC(w.prec, P, hipLaunchKernelGGL(k_multiaxpy<P>, dim3(pl.blocks), dim3(256), 0, c->stream,
                                              (const void*)base.p, stride, k, h, sgn, w.p, w.nrhs, pl,
                                              s.partial, n2 ? 1 : 0, overwrite ? 1 : 0));
  if (n2)
    hipLaunchKernelGGL(k_finalize_r, dim3(w.nrhs), dim3(64), 0, c->stream, s.partial,
                       (int)pl.blocks, 1, w.nrhs, n2);
  MGM_LAUNCH_CHECK();
}

// seg[g][o] = sum of data[o][j] over the g-th of G contiguous ranges of j
// (grid G x nout, fixed-order tree in LDS)
__global__ __launch_bounds__(256) void k_segment_sum(const double2* data, int64_t n, int nout, double2* seg) {
  const int g = blockIdx.x, G = gridDim.x, o = blockIdx.y;
  const int64_t per = (n + G - 1) / G, j0 = (int64_t)g * per, j1 = j0 + per < n ? j0 + per : n;
  double a = 0, b = 0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
    double2 v = data[(int64_t)o * n + j];
    a += v.x;
    b += v.y;
  }
  __shared__ double sa[256], sb[256];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) seg[(int64_t)g * nout + o] = make_double2(sa[0], sb[0]);
}

void b_finalize_dot_norm(Context* c, Scratch& s, const double2* part, int64_t nblk, int nrhs, double2* qr,
                         double* qq) {
  const int G = (int)std::min<int64_t>(64, std::max<int64_t>(1, nblk / 256));
  need(s, (size_t)G * 2 * nrhs);
  hipLaunchKernelGGL(k_segment_sum, dim3(G, 2 * nrhs), dim3(256), 0, c->stream, part, nblk, 2 * nrhs,
                     s.partial);
  hipLaunchKernelGGL(k_finalize_dn, dim3(2 * nrhs), dim3(64), 0, c->stream, s.partial, G, nrhs, qr, qq);
  MGM_LAUNCH_CHECK();
}

// One sweep of the re-orthogonalising Gram-Schmidt step: w <- w - sum_i h_i V_i
// and, from the same registers, out_i = V_i^H w (updated w), i < k <= kFusedGS.
// One sweep of w -= sum_i h_i V_i and a_i = V_i^H w (updated) for K basis
// vectors; K is a template parameter so registers and block-reduction rounds
// scale with the basis actually in use.
template <class P, int K>
__global__ __launch_bounds__(256) void k_multiaxpy_dot(const void* base, int64_t stride, const double2* h, void* w,
                                                       int nrhs, RedPlan pl, double2* partial) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double2 v[K];
#pragma unroll
  for (int i = 0; i < K; i++) v[i] = make_double2(0, 0);
  if (g < pl.J * nrhs) {
    const int r = (int)(g % nrhs);
    const int64_t j = g / nrhs;
    const typename P::S* B = (const typename P::S*)base;
    cx<double> hc[K], a[K];
#pragma unroll
    for (int i = 0; i < K; i++) {
      a[i] = {0, 0};
      const double2 hh = h[(int64_t)i * nrhs + r];
      hc[i] = {-hh.x, -hh.y};
    }
    for (int64_t m = j; m < pl.m; m += pl.J) {
      const int64_t e = m * nrhs + r;
      cx<double> wv = ldd<P>(w, e);
      cx<double> vv[K];
#pragma unroll
      for (int i = 0; i < K; i++) {
        vv[i] = ldd<P>(B + i * stride, e);
        fma_(wv, hc[i], vv[i]);
      }
      // the dots use the stored (rounded) value, rounded here in registers
      typename P::S st_;
      P::st(&st_, 0, cx<typename P::R>{(typename P::R)wv.re, (typename P::R)wv.im});
      const cx<typename P::R> wr = P::ld(&st_, 0);
      const cx<double> ws = {(double)wr.re, (double)wr.im};
      *((typename P::S*)w + e) = st_;
#pragma unroll
      for (int i = 0; i < K; i++) fmac_(a[i], vv[i], ws);
    }
#pragma unroll
    for (int i = 0; i < K; i++) v[i] = make_double2(a[i].re, a[i].im);
  }
  block_store<K>(v, partial, nrhs);
}

void b_multiaxpy_dot(Context* c, Scratch& s, Vec base, int64_t stride, int k, const double2* h, Vec w,
                     double2* out) {
  plain_layout(base);
  plain_layout(w);
  MGM_CHECK(k >= 1 && k <= kFusedGS, MGM_ERR_INVALID_ARG, "fused Gram-Schmidt sweep takes 1..16 vectors");
  RedPlan pl = red_plan(w.n(), w.nrhs);
  need(s, (size_t)pl.blocks * k * w.nrhs);
#define MGM_GS_CASE(KK)                                                                                      \
  case KK:                                                                                                   \
    DISPATCH_PREC(w.prec, P, hipLaunchKernelGGL((k_multiaxpy_dot<P, KK>), dim3(pl.blocks), dim3(256), 0,    \
                                                c->stream, (const void*)base.p, stride, h, w.p, w.nrhs, pl,   \
                                                s.partial));                                                  \
    break;
  switch (k) {
    MGM_GS_CASE(1) MGM_GS_CASE(2) MGM_GS_CASE(3) MGM_GS_CASE(4) MGM_GS_CASE(5) MGM_GS_CASE(6) MGM_GS_CASE(7)
    MGM_GS_CASE(8) MGM_GS_CASE(9) MGM_GS_CASE(10) MGM_GS_CASE(11) MGM_GS_CASE(12) MGM_GS_CASE(13)
    MGM_GS_CASE(14) MGM_GS_CASE(15) MGM_GS_CASE(16)
  }
#undef MGM_GS_CASE
  hipLaunchKernelGGL(k_finalize_c, dim3(k * w.nrhs), dim3(64), 0, c->stream, s.partial, (int)pl.blocks, k,
                     w.nrhs, k * w.nrhs, out, (int64_t)0);
  MGM_LAUNCH_CHECK();
}

// ----------------------------------------------------------- GMRES small

__global__ void kk_gmres_start(Givens G, const double* r2, int nrhs) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double b = sqrt(r2[r]);
  G.g[r] = make_double2(b, 0.0);
  for (int j = 1; j <= G.m; j++) G.g[(int64_t)j * nrhs + r] = make_double2(0, 0);
  G.est[r] = b;
}
void k_gmres_start(Context* c, Givens& G, const double* r2, int nrhs) {
  hipLaunchKernelGGL(kk_gmres_start, dim3(nblocks_for(nrhs, 64)), dim3(64), 0, c->stream, G, r2, nrhs);
  MGM_LAUNCH_CHECK();
}

// Complex Givens rotation with real cosine: for the pair (x, y),
// x' = c x + conj(s) y, y' = -s x + c y.  Chosen to zero y for (a, b):
// c = |a| / rho, s = b conj(a) / (|a| rho), rho = sqrt(|a|^2 + |b|^2).
__global__ void kk_gmres_column(Givens G, int j, const double* w2, int nrhs, int reorth) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const int m = G.m;
  cx<double> hcol[64];
  for (int i = 0; i <= j; i++) {
    double2 a = G.h[(int64_t)i * nrhs + r], b = reorth ? G.h2[(int64_t)i * nrhs + r] : make_double2(0, 0);
    hcol[i] = {a.x + b.x, a.y + b.y};
  }
  double beta = sqrt(w2[r]);
  G.beta[r] = beta;
  for (int i = 0; i < j; i++) {
    double cc = G.cs[(int64_t)i * nrhs + r];
    double2 s2 = G.sn[(int64_t)i * nrhs + r];
    cx<double> s = {s2.x, s2.y};
    cx<double> x = hcol[i], y = hcol[i + 1];
    hcol[i] = cc * x + cmulc(s, y);
    hcol[i + 1] = cc * y - s * x;
  }
  cx<double> a = hcol[j];
  double aa = sqrt(norm2(a));
  double rho = sqrt(aa * aa + beta * beta);
  double cc;
  cx<double> s, rjj;
  if (rho == 0.0) {
    cc = 1.0;
    s = {0, 0};
    rjj = {0, 0};
  } else if (aa == 0.0) {
    cc = 0.0;
    s = {1.0, 0.0};
    rjj = {beta, 0.0};
  } else {
    cc = aa / rho;
    s = (beta / (aa * rho)) * conj(a);
    rjj = (rho / aa) * a;
  }
  hcol[j] = rjj;
  G.cs[(int64_t)j * nrhs + r] = cc;
  G.sn[(int64_t)j * nrhs + r] = make_double2(s.re, s.im);
  for (int i = 0; i <= j; i++) G.R[((int64_t)j * m + i) * nrhs + r] = make_double2(hcol[i].re, hcol[i].im);
  double2 gj2 = G.g[(int64_t)j * nrhs + r];
  cx<double> gj = {gj2.x, gj2.y};
  cx<double> g1 = (-1.0) * (s * gj);
  gj = cc * gj;
  G.g[(int64_t)j * nrhs + r] = make_double2(gj.re, gj.im);
  G.g[(int64_t)(j + 1) * nrhs + r] = make_double2(g1.re, g1.im);
  G.est[r] = sqrt(norm2(g1));
}
void k_gmres_column(Context* c, Givens& G, int j, const double* w2, int nrhs, bool reorth) {
  MGM_CHECK(G.m <= 63, MGM_ERR_INVALID_ARG, "restart too long");
  hipLaunchKernelGGL(kk_gmres_column, dim3(nblocks_for(nrhs, 64)), dim3(64), 0, c->stream, G, j, w2, nrhs,
                     reorth ? 1 : 0);
  MGM_LAUNCH_CHECK();
}

__global__ void kk_gmres_solve(Givens G, int k, int nrhs) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const int m = G.m;
  for (int i = k - 1; i >= 0; i--) {
    double2 gi = G.g[(int64_t)i * nrhs + r];
    cx<double> acc = {gi.x, gi.y};
    for (int jj = i + 1; jj < k; jj++) {
      double2 Rij = G.R[((int64_t)jj * m + i) * nrhs + r];
      double2 yj = G.y[(int64_t)jj * nrhs + r];
      acc = acc - cx<double>{Rij.x, Rij.y} * cx<double>{yj.x, yj.y};
    }
    double2 Rii = G.R[((int64_t)i * m + i) * nrhs + r];
    double d = Rii.x * Rii.x + Rii.y * Rii.y;
    cx<double> yi = {0, 0};
    if (d > 0.0) yi = (1.0 / d) * cmulc(cx<double>{Rii.x, Rii.y}, acc);  // acc / Rii
    G.y[(int64_t)i * nrhs + r] = make_double2(yi.re, yi.im);
  }
}
void k_gmres_solve(Context* c, Givens& G, int k, int nrhs) {
  hipLaunchKernelGGL(kk_gmres_solve, dim3(nblocks_for(nrhs, 64)), dim3(64), 0, c->stream, G, k, nrhs);
  MGM_LAUNCH_CHECK();
}

}  // namespace mgm
