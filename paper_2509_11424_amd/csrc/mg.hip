// Aggregation-based transfers, block orthonormalisation of test vectors and
// the Galerkin coarse stencil (Sec. 2.2: R_l = P_l^H with unitary P_l,
// D_{l+1} = P_l^H D_l P_l).
#include "mg.h"

#include <type_traits>
#include "fine_dev.h"

namespace mgm {

// ----------------------------------------------------------------- geometry

LGeom coarse_geom(const LGeom& f, const int b[4], int ntv) {
  LGeom c;
  c.V = 1;
  for (int m = 0; m < 4; m++) {
    c.dims[m] = f.dims[m] / b[m];
    c.V *= c.dims[m];
  }
  c.dof = 2 * ntv;
  return c;
}

TGeom make_tgeom(const LGeom& f, const int b[4], int ntv) {
  TGeom t;
  t.f = f;
  for (int m = 0; m < 4; m++) t.b[m] = b[m];
  t.c = coarse_geom(f, b, ntv);
  t.ntv = ntv;
  t.bvol = b[0] * b[1] * b[2] * b[3];
  t.half = f.dof / 2;
  t.rows = t.bvol * t.half;
  return t;
}

__device__ __forceinline__ void coords_of(const LGeom& g, int64_t s, int c[4]) {
  c[0] = (int)(s % g.dims[0]); s /= g.dims[0];
  c[1] = (int)(s % g.dims[1]); s /= g.dims[1];
  c[2] = (int)(s % g.dims[2]); s /= g.dims[2];
  c[3] = (int)s;
}
__device__ __forceinline__ int64_t index_of(const LGeom& g, const int c[4]) {
  int x = (c[0] + g.dims[0]) % g.dims[0], y = (c[1] + g.dims[1]) % g.dims[1];
  int z = (c[2] + g.dims[2]) % g.dims[2], t = (c[3] + g.dims[3]) % g.dims[3];
  return x + (int64_t)g.dims[0] * (y + (int64_t)g.dims[1] * (z + (int64_t)g.dims[2] * t));
}
// fine site of local index loc inside aggregate a
__device__ __forceinline__ int64_t fine_site(const TGeom& t, int64_t a, int loc) {
  int ca[4], l[4], f[4];
  coords_of(t.c, a, ca);
  l[0] = loc % t.b[0]; loc /= t.b[0];
  l[1] = loc % t.b[1]; loc /= t.b[1];
  l[2] = loc % t.b[2]; loc /= t.b[2];
  l[3] = loc;
  for (int m = 0; m < 4; m++) f[m] = ca[m] * t.b[m] + l[m];
  return index_of(t.f, f);
}
// aggregate and local index of fine site s
__device__ __forceinline__ void agg_of(const TGeom& t, int64_t s, int64_t& a, int& loc) {
  int f[4], ca[4];
  coords_of(t.f, s, f);
  for (int m = 0; m < 4; m++) ca[m] = f[m] / t.b[m];
  a = index_of(t.c, ca);
  loc = (f[0] % t.b[0]) + t.b[0] * ((f[1] % t.b[1]) + t.b[1] * ((f[2] % t.b[2]) + t.b[2] * (f[3] % t.b[3])));
}

// ------------------------------------------------------------- agg map

__global__ void k_agg_map(TGeom t, int64_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = t.c.V * 2 * t.rows;
  if (i >= total) return;
  int row = (int)(i % t.rows);
  int64_t q = i / t.rows;
  int chi = (int)(q % 2);
  int64_t a = q / 2;
  int loc = row / t.half, j = row % t.half;
  int64_t s = fine_site(t, a, loc);
  out[i] = s * t.f.dof + chi * t.half + j;
}

void mg_agg_map(Context* c, const TGeom& t, int64_t* out) {
  int64_t total = t.c.V * 2 * t.rows;
  hipLaunchKernelGGL(k_agg_map, dim3(nblocks_for(total, 256)), dim3(256), 0, c->stream, t, out);
  MGM_LAUNCH_CHECK();
}

// ------------------------------------------------------------ transfers

// Transfers run one workgroup per (aggregate, chirality, rhs tile): the
// aggregate's P block (rows x N_tv) is streamed once through LDS in chunks of
// rows, so every P entry is read from HBM once per launch and reused by all
// right-hand sides of the tile.
constexpr int kTransferRT = 64;  // right-hand sides per workgroup
constexpr int kTransferLDS = 24576;  // bytes of streamed P rows (and restricted inputs)

__host__ __device__ inline int transfer_chunk_rows(int rows, int ntv, int rt, int cbytes, bool with_x) {
  const int per_row = (ntv + (with_x ? rt : 0)) * cbytes;
  int rc = kTransferLDS / per_row;
  if (rc > rows) rc = rows;
  return rc < 1 ? 1 : rc;
}

// fine sites of aggregate a, in local (lexicographic) order, into LDS
__device__ __forceinline__ void aggregate_sites(const TGeom& t, int64_t a, int64_t* sites) {
  int ca[4];
  coords_of(t.c, a, ca);
  for (int loc = threadIdx.x; loc < t.bvol; loc += blockDim.x) {
    int rem = loc, f[4];
#pragma unroll
    for (int m = 0; m < 4; m++) {
      const int l = rem % t.b[m];
      rem /= t.b[m];
      f[m] = ca[m] * t.b[m] + l;
    }
    sites[loc] = index_of(t.f, f);
  }
}

// P rows [row0, row0 + nr) of one (aggregate, chirality) block into LDS as
// complex R; FP16 blocks with K % 4 == 0 move 16 bytes (4 entries) per lane
template <class PM, typename R>
__device__ __forceinline__ void stage_p_rows(const typename PM::S* __restrict__ pb, int row0, int nr, int K,
                                             cx<R>* sP) {
  const int n = nr * K;
  if constexpr (std::is_same<PM, F16>::value) {
    if ((K & 3) == 0) {
      const uint4* src = reinterpret_cast<const uint4*>(pb + (int64_t)row0 * K);
      for (int i = threadIdx.x; i < n / 4; i += blockDim.x) {
        const uint4 v = src[i];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; e++) {
          __half2 h;
          __builtin_memcpy(&h, &w[e], 4);
          const float2 f = __half22float2(h);
          sP[4 * i + e] = {(R)f.x, (R)f.y};
        }
      }
      return;
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const cx<typename PM::R> v = PM::ld(pb, (int64_t)row0 * K + i);
    sP[i] = {(R)v.re, (R)v.im};
  }
}

// y_c[chi k][a][r] = sum_rows conj(P[a][chi][row][k]) x[chi half + j][site(loc)][r]
template <class P, class PM>
__global__ __launch_bounds__(256) void k_restrict(const typename P::S* __restrict__ x, typename P::S* __restrict__ yc,
                                                  const typename PM::S* __restrict__ Pm, TGeom t, int nrhs, int rc) {
  using R = typename P::R;
  extern __shared__ char smem[];
  const int64_t a = blockIdx.x >> 1;
  const int chi = blockIdx.x & 1;
  const int r0 = blockIdx.y * kTransferRT;
  const int rt = nrhs - r0 < kTransferRT ? nrhs - r0 : kTransferRT;
  const int K = t.ntv, half = t.half, rows = t.rows;
  const int64_t Vc = t.c.V, Vf = t.f.V;
  int64_t* sS = reinterpret_cast<int64_t*>(smem);                      // [bvol] fine sites
  cx<R>* sP = reinterpret_cast<cx<R>*>(smem + (size_t)t.bvol * 8);     // [rc][K]
  cx<R>* sX = sP + (size_t)rc * K;                                      // [rc][rt]
  const int O = K * rt;                          // outputs of this workgroup, r fastest
  aggregate_sites(t, a, sS);
  __syncthreads();
  constexpr int MAXO = (32 * kTransferRT + 255) / 256;
  cx<R> acc[MAXO];
#pragma unroll
  for (int m = 0; m < MAXO; m++) acc[m] = {0, 0};
  const typename PM::S* pb = Pm + ((a * 2 + chi) * rows) * (int64_t)K;
  for (int row0 = 0; row0 < rows; row0 += rc) {
    const int nr = rows - row0 < rc ? rows - row0 : rc;
    stage_p_rows<PM, R>(pb, row0, nr, K, sP);
    for (int i = threadIdx.x; i < nr * rt; i += blockDim.x) {
      const int ii = i / rt, r = i - ii * rt;
      const int row = row0 + ii, loc = row / half, j = row - loc * half;
      sX[i] = P::ld(x, ((int64_t)(chi * half + j) * Vf + sS[loc]) * nrhs + r0 + r);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXO; m++) {
      const int o = threadIdx.x + m * 256;
      if (o < O) {
        const int k = o / rt, r = o - k * rt;
        // four independent partial sums keep several LDS reads in flight
        cx<R> s0 = acc[m], s1 = {0, 0}, s2 = {0, 0}, s3 = {0, 0};
        int i = 0;
        for (; i + 4 <= nr; i += 4) {
          fmac_(s0, sP[i * K + k], sX[i * rt + r]);
          fmac_(s1, sP[(i + 1) * K + k], sX[(i + 1) * rt + r]);
          fmac_(s2, sP[(i + 2) * K + k], sX[(i + 2) * rt + r]);
          fmac_(s3, sP[(i + 3) * K + k], sX[(i + 3) * rt + r]);
        }
        for (; i < nr; i++) fmac_(s0, sP[i * K + k], sX[i * rt + r]);
        acc[m] = (s0 + s1) + (s2 + s3);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < MAXO; m++) {
    const int o = threadIdx.x + m * 256;
    if (o < O) {
      const int k = o / rt, r = o - k * rt;
      P::st(yc, ((int64_t)(chi * K + k) * Vc + a) * nrhs + r0 + r, acc[m]);
    }
  }
}

// y = P x_c (mode 0), x - P x_c (mode 1), y + P x_c (mode 2)
template <class P, class PM>
__global__ __launch_bounds__(256) void k_prolong(const typename P::S* __restrict__ xc, const typename P::S* __restrict__ x,
                                                 typename P::S* __restrict__ y, const typename PM::S* __restrict__ Pm,
                                                 TGeom t, int nrhs, int mode, int rc) {
  using R = typename P::R;
  extern __shared__ char smem[];
  const int64_t a = blockIdx.x >> 1;
  const int chi = blockIdx.x & 1;
  const int r0 = blockIdx.y * kTransferRT;
  const int rt = nrhs - r0 < kTransferRT ? nrhs - r0 : kTransferRT;
  const int K = t.ntv, half = t.half, rows = t.rows;
  const int64_t Vc = t.c.V, Vf = t.f.V;
  int64_t* sS = reinterpret_cast<int64_t*>(smem);                      // [bvol] fine sites
  cx<R>* sC = reinterpret_cast<cx<R>*>(smem + (size_t)t.bvol * 8);     // [K][rt] coarse values
  cx<R>* sP = sC + (size_t)K * rt;                                      // [rc][K]
  aggregate_sites(t, a, sS);
  for (int i = threadIdx.x; i < K * rt; i += blockDim.x) {
    const int k = i / rt, r = i - k * rt;
    sC[i] = P::ld(xc, ((int64_t)(chi * K + k) * Vc + a) * nrhs + r0 + r);
  }
  const typename PM::S* pb = Pm + ((a * 2 + chi) * rows) * (int64_t)K;
  for (int row0 = 0; row0 < rows; row0 += rc) {
    const int nr = rows - row0 < rc ? rows - row0 : rc;
    __syncthreads();  // previous chunk consumed (and sC written on the first pass)
    stage_p_rows<PM, R>(pb, row0, nr, K, sP);
    __syncthreads();
    for (int o = threadIdx.x; o < nr * rt; o += blockDim.x) {
      const int ii = o / rt, r = o - ii * rt;
      cx<R> a0 = {0, 0}, a1 = {0, 0}, a2 = {0, 0}, a3 = {0, 0};
      int k = 0;
      for (; k + 4 <= K; k += 4) {
        fma_(a0, sP[ii * K + k], sC[k * rt + r]);
        fma_(a1, sP[ii * K + k + 1], sC[(k + 1) * rt + r]);
        fma_(a2, sP[ii * K + k + 2], sC[(k + 2) * rt + r]);
        fma_(a3, sP[ii * K + k + 3], sC[(k + 3) * rt + r]);
      }
      for (; k < K; k++) fma_(a0, sP[ii * K + k], sC[k * rt + r]);
      cx<R> acc = (a0 + a1) + (a2 + a3);
      const int row = row0 + ii, loc = row / half, j = row - loc * half;
      const int64_t e = ((int64_t)(chi * half + j) * Vf + sS[loc]) * nrhs + r0 + r;
      if (mode == 1) acc = P::ld(x, e) - acc;
      else if (mode == 2) acc = P::ld(y, e) + acc;
      P::st(y, e, acc);
    }
  }
}

double Transfer::bytes(mgm_prec p, int nrhs) const {
  double w = (double)prec_bytes(p);
  return (double)t.c.V * 2 * t.rows * t.ntv * w + (double)t.f.V * t.f.dof * nrhs * w +
         (double)t.c.V * t.c.dof * nrhs * w;
}

void Transfer::restrict_(mgm_prec p, const void* x, void* yc, int nrhs) const {
  ProfScope ps(ctx, KC_TRANSFER, bytes(p, nrhs));
  const dim3 nb((unsigned)(2 * t.c.V), (unsigned)((nrhs + kTransferRT - 1) / kTransferRT)), tb(256);
  const int rt = nrhs < kTransferRT ? nrhs : kTransferRT;
  MGM_CHECK(t.ntv <= 32 && t.bvol <= 1024, MGM_ERR_SHAPE,
            "transfers support at most 32 test vectors and 1024 sites per aggregate");
  if (p == MGM_PREC_F64) {
    const int rc = transfer_chunk_rows(t.rows, t.ntv, rt, 16, true);
    hipLaunchKernelGGL((k_restrict<F64, F64>), nb, tb, (size_t)t.bvol * 8 + (size_t)rc * (t.ntv + rt) * 16, ctx->stream,
                       (const double2*)x, (double2*)yc, P64, t, nrhs, rc);
  } else if (p == MGM_PREC_F32) {
    const int rc = transfer_chunk_rows(t.rows, t.ntv, rt, 8, true);
    hipLaunchKernelGGL((k_restrict<F32, F16>), nb, tb, (size_t)t.bvol * 8 + (size_t)rc * (t.ntv + rt) * 8, ctx->stream,
                       (const float2*)x, (float2*)yc, P16, t, nrhs, rc);
  } else {
    throw Error(MGM_ERR_INVALID_ARG, "restrict: precision must be F64 or F32");
  }
  MGM_LAUNCH_CHECK();
}

void Transfer::prolong(mgm_prec p, const void* xc, const void* x, void* y, int nrhs, int mode) const {
  ProfScope ps(ctx, KC_TRANSFER, bytes(p, nrhs));
  const dim3 nb((unsigned)(2 * t.c.V), (unsigned)((nrhs + kTransferRT - 1) / kTransferRT)), tb(256);
  const int rt = nrhs < kTransferRT ? nrhs : kTransferRT;
  MGM_CHECK(t.ntv <= 32 && t.bvol <= 1024, MGM_ERR_SHAPE,
            "transfers support at most 32 test vectors and 1024 sites per aggregate");
  if (p == MGM_PREC_F64) {
    const int rc = transfer_chunk_rows(t.rows, t.ntv, rt, 16, false);
    hipLaunchKernelGGL((k_prolong<F64, F64>), nb, tb, (size_t)t.bvol * 8 + ((size_t)t.ntv * rt + (size_t)rc * t.ntv) * 16, ctx->stream,
                       (const double2*)xc, (const double2*)x, (double2*)y, P64, t, nrhs, mode, rc);
  } else if (p == MGM_PREC_F32) {
    const int rc = transfer_chunk_rows(t.rows, t.ntv, rt, 8, false);
    hipLaunchKernelGGL((k_prolong<F32, F16>), nb, tb, (size_t)t.bvol * 8 + ((size_t)t.ntv * rt + (size_t)rc * t.ntv) * 8, ctx->stream,
                       (const float2*)xc, (const float2*)x, (float2*)y, P16, t, nrhs, mode, rc);
  } else {
    throw Error(MGM_ERR_INVALID_ARG, "prolong: precision must be F64 or F32");
  }
  MGM_LAUNCH_CHECK();
}

// ------------------------------------------------------------ block QR

__device__ double2 block_sum2(double2 v, double2* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = make_double2(red[t].x + red[t + s].x, red[t].y + red[t + s].y);
    __syncthreads();
  }
  double2 out = red[0];
  __syncthreads();
  return out;
}

// Modified Gram-Schmidt over the columns of every (aggregate, chirality)
// block, each column orthogonalised twice against the previous ones.
__global__ void k_block_mgs2(const double2* __restrict__ tv, double2* __restrict__ Pm, TGeom t, int* flag) {
  extern __shared__ double2 w[];
  __shared__ double2 red[256];
  const int64_t a = blockIdx.x >> 1;
  const int chi = blockIdx.x & 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ntv = t.ntv;
  double2* Pb = Pm + (a * 2 + chi) * (int64_t)t.rows * ntv;
  for (int k = 0; k < ntv; k++) {
    double n0 = 0;
    for (int row = tid; row < t.rows; row += nt) {
      int loc = row / t.half, j = row % t.half;
      int64_t s = fine_site(t, a, loc);
      double2 v = tv[((int64_t)(chi * t.half + j) * t.f.V + s) * ntv + k];
      w[row] = v;
      n0 += v.x * v.x + v.y * v.y;
    }
    n0 = block_sum2(make_double2(n0, 0), red).x;
    for (int pass = 0; pass < 2; pass++)
      for (int jj = 0; jj < k; jj++) {
        cx<double> h = {0, 0};
        for (int row = tid; row < t.rows; row += nt) {
          double2 qv = Pb[(int64_t)row * ntv + jj];
          fmac_(h, cx<double>{qv.x, qv.y}, cx<double>{w[row].x, w[row].y});
        }
        double2 hs = block_sum2(make_double2(h.re, h.im), red);
        for (int row = tid; row < t.rows; row += nt) {
          double2 qv = Pb[(int64_t)row * ntv + jj];
          cx<double> wv = {w[row].x, w[row].y};
          wv = wv - cx<double>{hs.x, hs.y} * cx<double>{qv.x, qv.y};
          w[row] = make_double2(wv.re, wv.im);
        }
        __syncthreads();
      }
    double nn = 0;
    for (int row = tid; row < t.rows; row += nt) nn += w[row].x * w[row].x + w[row].y * w[row].y;
    nn = block_sum2(make_double2(nn, 0), red).x;
    double nrm = sqrt(nn);
    double inv = 1.0 / nrm;
    if (!(n0 > 0.0) || !(nrm >= 1e-12 * sqrt(n0))) {
      inv = 0.0;
      if (tid == 0) *flag = 1;
    }
    for (int row = tid; row < t.rows; row += nt)
      Pb[(int64_t)row * ntv + k] = make_double2(w[row].x * inv, w[row].y * inv);
    __syncthreads();
  }
}

void mg_block_mgs2(Context* c, const TGeom& t, const double2* tv, double2* P, int* flag) {
  size_t sh = (size_t)t.rows * sizeof(double2);
  MGM_CHECK(sh <= 64 * 1024, MGM_ERR_SHAPE, "aggregate too large for LDS column");
  hipLaunchKernelGGL(k_block_mgs2, dim3((unsigned)(t.c.V * 2)), dim3(256), sh, c->stream, tv, P, t, flag);
  MGM_LAUNCH_CHECK();
}

// ------------------------------------------------------------ Galerkin

// Which stencil direction of the aggregate a fine hop k from local
// coordinates l contributes to (0 when it stays inside).
__device__ __forceinline__ int hop_target(int k, const int l[4], const int b[4]) {
  if (k == 0) return 0;
  int mu = (k - 1) & 3;
  if (k <= 4) return l[mu] == b[mu] - 1 ? k : 0;
  return l[mu] == 0 ? k : 0;
}

// One Wilson-clover block of D (12 x 12 at site s, direction k) applied to a
// single spinor p; y is the neighbour site of the hop.
__device__ void wilson_block(const FineOp& op, int k, int64_t s, int64_t y, const int fc[4],
                             const cx<double>* p, cx<double>* out) {
  const Geom& g = op.g;
  if (k == 0) {
    clover_block<F64>(op.C64, g.V, s, 0, p, out);
    clover_block<F64>(op.C64, g.V, s, 1, p + 6, out + 6);
    return;
  }
  const bool fwd = k <= 4;
  const int mu = (k - 1) & 3;
  const int ext[4] = {g.X, g.Y, g.Z, g.T};
  double ph = 1.0;
  if (mu == 3 && g.antiperiodic && ((fwd && fc[3] == ext[3] - 1) || (!fwd && fc[3] == 0))) ph = -1.0;
  const int64_t ls = fwd ? s : y;  // site owning the link U_mu
  cx<double> U[3][3];
  for (int q = 0; q < 9; q++) {
    double2 v = op.U64[(int64_t)(mu * 9 + q) * g.V + ls];
    U[q / 3][q % 3] = {v.x, v.y};
  }
  cx<double> h[2][3];
  for (int a = 0; a < 3; a++) {
    cx<double> a0, a1;
    A_times(mu, p[6 + a], p[9 + a], a0, a1);
    h[0][a] = fwd ? p[a] - a0 : p[a] + a0;
    h[1][a] = fwd ? p[3 + a] - a1 : p[3 + a] + a1;
  }
  const double f = -0.5 * ph;
  for (int a = 0; a < 3; a++) {
    cx<double> g0 = {0, 0}, g1 = {0, 0};
    for (int b = 0; b < 3; b++) {
      if (fwd) {
        fma_(g0, U[a][b], h[0][b]);
        fma_(g1, U[a][b], h[1][b]);
      } else {
        fmac_(g0, U[b][a], h[0][b]);
        fmac_(g1, U[b][a], h[1][b]);
      }
    }
    g0 = f * g0;
    g1 = f * g1;
    cx<double> d0, d1;
    Ad_times(mu, g0, g1, d0, d1);
    out[a] = g0;
    out[3 + a] = g1;
    out[6 + a] = fwd ? (-1.0) * d0 : d0;
    out[9 + a] = fwd ? (-1.0) * d1 : d1;
  }
}

__device__ __forceinline__ int64_t hop_neighbour(const LGeom& g, const int c[4], int k) {
  if (k == 0) return index_of(g, c);
  int mu = (k - 1) & 3;
  int cc[4] = {c[0], c[1], c[2], c[3]};
  cc[mu] += (k <= 4) ? 1 : -1;
  return index_of(g, cc);
}

constexpr int kGalPairs = 16;  // (i, j) pairs per thread: d*d <= 256*16

__global__ void k_galerkin_fine(FineOp op, TGeom t, const double2* __restrict__ Pm, double2* __restrict__ Ac) {
  extern __shared__ double2 T[];  // [12][d]
  const int64_t a = blockIdx.x;
  const int tgt = blockIdx.y;
  const int d = 2 * t.ntv, ntv = t.ntv, tid = threadIdx.x;
  cx<double> acc[kGalPairs];
  for (int q = 0; q < kGalPairs; q++) acc[q] = {0, 0};
  int ca[4];
  coords_of(t.c, a, ca);
  for (int loc = 0; loc < t.bvol; loc++) {
    int l[4], rem = loc, fc[4];
    l[0] = rem % t.b[0]; rem /= t.b[0];
    l[1] = rem % t.b[1]; rem /= t.b[1];
    l[2] = rem % t.b[2]; rem /= t.b[2];
    l[3] = rem;
    for (int m = 0; m < 4; m++) fc[m] = ca[m] * t.b[m] + l[m];
    const int64_t s = index_of(t.f, fc);
    for (int k = 0; k < 9; k++) {
      if (hop_target(k, l, t.b) != tgt) continue;
      const int64_t y = hop_neighbour(t.f, fc, k);
      if (tid < d) {
        const int j = tid, chij = j / ntv, kk = j % ntv;
        int64_t ay;
        int locy;
        agg_of(t, y, ay, locy);
        cx<double> p[12];
        for (int m = 0; m < 12; m++) p[m] = {0, 0};
        for (int m = 0; m < 6; m++) {
          double2 v = Pm[((ay * 2 + chij) * t.rows + locy * 6 + m) * (int64_t)ntv + kk];
          p[6 * chij + m] = {v.x, v.y};
        }
        cx<double> o[12];
        wilson_block(op, k, s, y, fc, p, o);
        for (int m = 0; m < 12; m++) T[m * d + j] = make_double2(o[m].re, o[m].im);
      }
      __syncthreads();
      for (int q = 0; q < kGalPairs; q++) {
        int pidx = tid + q * blockDim.x;
        if (pidx >= d * d) break;
        int i = pidx / d, j = pidx % d;
        int chii = i / ntv, ki = i % ntv;
        const double2* pr = Pm + ((a * 2 + chii) * t.rows + loc * 6) * (int64_t)ntv + ki;
        for (int m = 0; m < 6; m++) {
          double2 pv = pr[(int64_t)m * ntv];
          double2 tv = T[(6 * chii + m) * d + j];
          fmac_(acc[q], cx<double>{pv.x, pv.y}, cx<double>{tv.x, tv.y});
        }
      }
      __syncthreads();
    }
  }
  const int64_t Vc = t.c.V;
  for (int q = 0; q < kGalPairs; q++) {
    int pidx = tid + q * blockDim.x;
    if (pidx >= d * d) break;
    int i = pidx / d, j = pidx % d;
    Ac[((int64_t)(tgt * d + i) * d + j) * Vc + a] = make_double2(acc[q].re, acc[q].im);
  }
}

__global__ void k_galerkin_coarse(CoarseOp op, TGeom t, const double2* __restrict__ Pm, double2* __restrict__ Ac) {
  extern __shared__ double2 T[];  // [dl][d]
  const int64_t a = blockIdx.x;
  const int tgt = blockIdx.y;
  const int d = 2 * t.ntv, ntv = t.ntv, tid = threadIdx.x;
  const int dl = t.f.dof, hl = t.half;
  const int64_t Vl = t.f.V;
  cx<double> acc[kGalPairs];
  for (int q = 0; q < kGalPairs; q++) acc[q] = {0, 0};
  int ca[4];
  coords_of(t.c, a, ca);
  for (int loc = 0; loc < t.bvol; loc++) {
    int l[4], rem = loc, fc[4];
    l[0] = rem % t.b[0]; rem /= t.b[0];
    l[1] = rem % t.b[1]; rem /= t.b[1];
    l[2] = rem % t.b[2]; rem /= t.b[2];
    l[3] = rem;
    for (int m = 0; m < 4; m++) fc[m] = ca[m] * t.b[m] + l[m];
    const int64_t s = index_of(t.f, fc);
    for (int k = 0; k < 9; k++) {
      if (hop_target(k, l, t.b) != tgt) continue;
      const int64_t y = hop_neighbour(t.f, fc, k);
      if (tid < d) {
        const int j = tid, chij = j / ntv, kk = j % ntv;
        int64_t ay;
        int locy;
        agg_of(t, y, ay, locy);
        const double2* py = Pm + ((ay * 2 + chij) * t.rows + locy * hl) * (int64_t)ntv + kk;
        for (int i2 = 0; i2 < dl; i2++) {
          cx<double> o = {0, 0};
          const double2* Arow = op.A64 + ((int64_t)(k * dl + i2) * dl + chij * hl) * Vl + s;
          for (int mm = 0; mm < hl; mm++) {
            double2 av = Arow[(int64_t)mm * Vl];
            double2 pv = py[(int64_t)mm * ntv];
            fma_(o, cx<double>{av.x, av.y}, cx<double>{pv.x, pv.y});
          }
          T[i2 * d + j] = make_double2(o.re, o.im);
        }
      }
      __syncthreads();
      for (int q = 0; q < kGalPairs; q++) {
        int pidx = tid + q * blockDim.x;
        if (pidx >= d * d) break;
        int i = pidx / d, j = pidx % d;
        int chii = i / ntv, ki = i % ntv;
        const double2* pr = Pm + ((a * 2 + chii) * t.rows + loc * hl) * (int64_t)ntv + ki;
        for (int mm = 0; mm < hl; mm++) {
          double2 pv = pr[(int64_t)mm * ntv];
          double2 tv = T[(chii * hl + mm) * d + j];
          fmac_(acc[q], cx<double>{pv.x, pv.y}, cx<double>{tv.x, tv.y});
        }
      }
      __syncthreads();
    }
  }
  const int64_t Vc = t.c.V;
  for (int q = 0; q < kGalPairs; q++) {
    int pidx = tid + q * blockDim.x;
    if (pidx >= d * d) break;
    int i = pidx / d, j = pidx % d;
    Ac[((int64_t)(tgt * d + i) * d + j) * Vc + a] = make_double2(acc[q].re, acc[q].im);
  }
}

void mg_galerkin_fine(Context* c, const FineOp& op, const Transfer& T, CoarseOp& out) {
  const TGeom& t = T.t;
  const int d = 2 * t.ntv;
  MGM_CHECK(d * d <= 256 * kGalPairs && d <= 64, MGM_ERR_SHAPE, "too many test vectors");
  size_t sh = (size_t)12 * d * sizeof(double2);
  hipLaunchKernelGGL(k_galerkin_fine, dim3((unsigned)t.c.V, 9), dim3(256), sh, c->stream, op, t, T.P64, out.A64);
  MGM_LAUNCH_CHECK();
}

void mg_galerkin_coarse(Context* c, const CoarseOp& op, const Transfer& T, CoarseOp& out) {
  const TGeom& t = T.t;
  const int d = 2 * t.ntv;
  MGM_CHECK(d * d <= 256 * kGalPairs && d <= 64 && t.f.dof <= 64, MGM_ERR_SHAPE, "too many test vectors");
  size_t sh = (size_t)t.f.dof * d * sizeof(double2);
  hipLaunchKernelGGL(k_galerkin_coarse, dim3((unsigned)t.c.V, 9), dim3(256), sh, c->stream, op, t, T.P64,
                     out.A64);
  MGM_LAUNCH_CHECK();
}

// ------------------------------------------------------- coarse stencil

// y(s) = sum_dir A[dir](s) x(nbr(s, dir)) runs on the matrix cores
// (coarse_mfma.hip): FP64 and FP32 with 16x16x4 MFMAs, BF16 operands with
// FP32 accumulation for the mixed-precision preconditioner.

double CoarseOp::bytes(mgm_prec p, int nrhs) const {
  // algorithmic bytes: nine complex d x d blocks once, x and y once
  double wa = p == MGM_PREC_F64 ? 16.0 : p == MGM_PREC_F32 ? 8.0 : 4.0;
  double wv = p == MGM_PREC_F64 ? 16.0 : 8.0;
  return (double)g.V * (9.0 * d * d * wa + 2.0 * d * nrhs * wv);
}

void CoarseOp::apply(mgm_prec p, const void* x, void* y, int nrhs) const {
  if (p == MGM_PREC_F64) {
    coarse_apply_mfma64(*this, (const double2*)x, (double2*)y, nrhs);
  } else if (p == MGM_PREC_F32) {
    MGM_CHECK(A32 != nullptr, MGM_ERR_INVALID_ARG, "FP32 coarse stencil not built (mixed == 0)");
    coarse_apply_mfma32(*this, (const float2*)x, (float2*)y, nrhs);
  } else if (p == MGM_PREC_BF16) {
    coarse_apply_mfma(*this, (const float2*)x, (float2*)y, nrhs);
  } else {
    throw Error(MGM_ERR_INVALID_ARG, "coarse apply: unsupported precision");
  }
}

// ---------------------------------------------------------- conversions

// P entries are O(1/sqrt(rows)), well inside the FP16 range
__global__ void k_c64_to_c16(__half2* o, const double2* in, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = __floats2half2_rn((float)in[i].x, (float)in[i].y);
}

void mg_convert_P(Context* c, Transfer& T) {
  int64_t n = T.t.c.V * 2 * (int64_t)T.t.rows * T.t.ntv;
  hipLaunchKernelGGL(k_c64_to_c16, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, T.P16, T.P64, n);
  MGM_LAUNCH_CHECK();
}

void mg_convert_A(Context* c, CoarseOp& A) { mg_mfma32_pack(c, A); }

}  // namespace mgm
