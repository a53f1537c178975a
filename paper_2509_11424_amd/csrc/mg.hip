// Aggregation-based transfers, block orthonormalisation of test vectors and
// the Galerkin coarse stencil (Sec. 2.2: R_l = P_l^H with unitary P_l,
// D_{l+1} = P_l^H D_l P_l).
#include "mg.h"

#include <type_traits>
#include "fine_dev.h"
#include "group.h"

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
// right-hand sides of the tile.  Each thread owns a 4 x 4 register tile of
// the block's products (four test vectors or rows by four right-hand sides),
// so one pair of 32-byte LDS reads feeds sixteen complex FMAs.
constexpr int kTransferRT = 64;     // right-hand sides per workgroup
constexpr int kTransferTB = 256;    // threads per workgroup
constexpr int kRestrictLDS = 24576; // bytes of streamed P rows and restricted inputs
constexpr int kProlongLDS = 24576;  // bytes of streamed (transposed) P rows

__host__ __device__ inline int round4(int v) { return (v + 3) & ~3; }
__host__ __device__ inline int sites_bytes(int bvol) { return (bvol * 8 + 15) & ~15; }

// restrict: the rhs tile of width rt splits into T = (Kp/4)(rtp/4) output
// tiles; G = 256 / T thread groups share the rows of a chunk
__host__ __device__ inline int restrict_groups(int K, int rt) { return kTransferTB / ((round4(K) / 4) * (round4(rt) / 4)); }

// rows per chunk: the fewest equal chunks that fit the byte budget, rounded
// up to a multiple of `mult` when that still fits
inline int balanced_chunk(int rows, int rc_max, int mult) {
  if (rc_max < 1) rc_max = 1;
  if (rc_max >= rows) return rows;
  const int n = (rows + rc_max - 1) / rc_max;
  int rc = (rows + n - 1) / n;
  const int up = (rc + mult - 1) / mult * mult;
  return up <= rc_max ? up : rc;
}

inline int restrict_chunk_rows(const TGeom& t, int rt, int cbytes) {
  const int Kp = round4(t.ntv), rtp = round4(rt);
  return balanced_chunk(t.rows, kRestrictLDS / ((Kp + rtp) * cbytes), restrict_groups(t.ntv, rt));
}
inline size_t restrict_lds(const TGeom& t, int rt, int rc, int cbytes) {
  const size_t chunk = (size_t)rc * (round4(t.ntv) + round4(rt)) * cbytes;
  const size_t red = (size_t)kTransferTB * 4 * cbytes;
  return sites_bytes(t.bvol) + (chunk > red ? chunk : red);
}
// prolong: TI rows per thread, chunks of about one tile per thread (at
// most kProlongLDS bytes of P), rows a multiple of TI
inline int prolong_chunk_rows(const TGeom& t, int rt, int cbytes, int TI) {
  const int ntr = round4(rt) / 4;
  const int want = TI * ((kTransferTB + ntr - 1) / ntr);
  int cap = kProlongLDS / (t.ntv * cbytes);
  cap = (cap < want ? cap : want) / TI * TI;
  if (cap < TI) cap = TI;
  const int rows = (t.rows + TI - 1) / TI * TI;
  const int rc = balanced_chunk(rows, cap, TI);
  return (rc + TI - 1) / TI * TI;
}
inline size_t prolong_lds(const TGeom& t, int rt, int rc, int cbytes) {
  return sites_bytes(t.bvol) + ((size_t)t.ntv * round4(rt) + (size_t)rc * t.ntv) * cbytes;
}
// rhs per prolongation workgroup: kTransferRT, halved while the coarse
// values of a full tile would take more than half of the 64 KiB LDS (FP64
// with more than 32 test vectors, FP32 with more than 64)
inline int prolong_rt(const TGeom& t, int cbytes) {
  int rt = kTransferRT;
  while (rt > 4 && (size_t)t.ntv * rt * cbytes > 32768) rt /= 2;
  return rt;
}
// rhs per restriction workgroup: kTransferRT, halved while the 4 x 4 output
// tiles of (test vectors) x (rhs) outnumber the workgroup's threads (more
// than 64 test vectors)
inline int restrict_rt(const TGeom& t) {
  int rt = kTransferRT;
  while (rt > 4 && (round4(t.ntv) / 4) * (rt / 4) > kTransferTB) rt /= 2;
  return rt;
}

// fine sites of aggregate a, in local (lexicographic) order, into LDS
__device__ __forceinline__ void aggregate_sites(const TGeom& t, int64_t a, int64_t* sites) {
  int ca[4];
  coords_of(t.c, a, ca);
  for (int loc = threadIdx.x; loc < t.bvol; loc += kTransferTB) {
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
// complex R: entry (row ii, vector k) goes to sP[ii * ld + k] (row-major,
// columns K..ld-1 zeroed) or, transposed, to sP[k * ld + ii].  FP16 blocks
// with K % 4 == 0 move 16 bytes (4 entries) per lane.
template <class PM, typename R, bool TRANS>
__device__ __forceinline__ void stage_p_rows(const typename PM::S* __restrict__ pb, int row0, int nr, int K, int ld,
                                             cx<R>* sP) {
  if constexpr (std::is_same<PM, F16>::value) {
    if ((K & 3) == 0) {
      const int K4 = K >> 2;
      const uint4* src = reinterpret_cast<const uint4*>(pb + (int64_t)row0 * K);
      for (int i = threadIdx.x; i < nr * K4; i += kTransferTB) {
        const uint4 v = src[i];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        const int ii = i / K4, k0 = (i - ii * K4) * 4;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          __half2 h;
          __builtin_memcpy(&h, &w[e], 4);
          const float2 f = __half22float2(h);
          if (TRANS)
            sP[(k0 + e) * ld + ii] = {(R)f.x, (R)f.y};
          else
            sP[ii * ld + k0 + e] = {(R)f.x, (R)f.y};  // ld == K here
        }
      }
      return;
    }
  }
  if (TRANS) {
    for (int i = threadIdx.x; i < nr * K; i += kTransferTB) {
      const int ii = i / K, k = i - ii * K;
      const cx<typename PM::R> v = PM::ld(pb, (int64_t)row0 * K + i);
      sP[k * ld + ii] = {(R)v.re, (R)v.im};
    }
  } else {
    for (int i = threadIdx.x; i < nr * ld; i += kTransferTB) {
      const int ii = i / ld, k = i - ii * ld;
      cx<R> v = {0, 0};
      if (k < K) {
        const cx<typename PM::R> u = PM::ld(pb, (int64_t)(row0 + ii) * K + k);
        v = {(R)u.re, (R)u.im};
      }
      sP[i] = v;
    }
  }
}

// four consecutive complex entries from 16-byte aligned LDS
template <typename R>
__device__ __forceinline__ void lds_ld4(const cx<R>* p, cx<R> (&v)[4]) {
  if constexpr (std::is_same<R, float>::value) {
    const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
    v[0] = {a.x, a.y};
    v[1] = {a.z, a.w};
    v[2] = {b.x, b.y};
    v[3] = {b.z, b.w};
  } else {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const double2 a = reinterpret_cast<const double2*>(p)[j];
      v[j] = {a.x, a.y};
    }
  }
}

// y_c[chi k][a][r] = sum_rows conj(P[a][chi][row][k]) x[chi half + j][site(loc)][r]
// Thread (g, u) accumulates the output tile u = (k/4, r/4) over the rows
// g, g + G, ... of every chunk; the G partial tiles are then summed in group
// order through LDS.
// The input x may be stored in another format PX, scaled per rhs by xs, and
// in column groups of xgs right-hand sides (xgs = nrhs: plain layout).
template <class P, class PM, class PX = P>
__global__ __launch_bounds__(256) void k_restrict(const typename PX::S* __restrict__ x, typename P::S* __restrict__ yc,
                                                  const typename PM::S* __restrict__ Pm, TGeom t, int nrhs, int rc,
                                                  int rtile, const double* __restrict__ xs, int xgs) {
  using R = typename P::R;
  extern __shared__ __align__(16) char smem[];
  const int64_t a = blockIdx.x >> 1;
  const int chi = blockIdx.x & 1;
  const int r0 = blockIdx.y * rtile;
  const int rt = nrhs - r0 < rtile ? nrhs - r0 : rtile;
  const int K = t.ntv, half = t.half, rows = t.rows;
  const int Kp = round4(K), rtp = round4(rt), ntr = rtp >> 2;
  const int T = (Kp >> 2) * ntr, G = kTransferTB / T;
  const int64_t Vc = t.c.V, Vf = t.f.V;
  const int tid = threadIdx.x;
  const bool active = tid < G * T;
  const int g = tid / T, u = tid - g * T;
  const int kt = u / ntr, rtt = u - kt * ntr;
  int64_t* sS = reinterpret_cast<int64_t*>(smem);                        // [bvol] fine sites
  cx<R>* sP = reinterpret_cast<cx<R>*>(smem + sites_bytes(t.bvol));      // [rc][Kp]
  cx<R>* sX = sP + (size_t)rc * Kp;                                       // [rc][rtp]
  aggregate_sites(t, a, sS);
  __syncthreads();
  cx<R> acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = {0, 0};
  const typename PM::S* pb = Pm + ((a * 2 + chi) * rows) * (int64_t)K;
  for (int row0 = 0; row0 < rows; row0 += rc) {
    const int nr = rows - row0 < rc ? rows - row0 : rc;
    stage_p_rows<PM, R, false>(pb, row0, nr, K, Kp, sP);
    for (int i = tid; i < nr * rtp; i += kTransferTB) {
      const int ii = i / rtp, r = i - ii * rtp;
      cx<R> v = {0, 0};
      if (r < rt) {
        const int row = row0 + ii, loc = row / half, j = row - loc * half;
        const cx<typename PX::R> u =
            PX::ld(x, grouped_index((int64_t)(chi * half + j) * Vf + sS[loc], r0 + r, nrhs, xgs, 2 * half * Vf));
        v = {(R)u.re, (R)u.im};
        if (xs) v = (R)xs[r0 + r] * v;
      }
      sX[i] = v;
    }
    __syncthreads();
    if (active) {
      for (int i = g; i < nr; i += G) {
        cx<R> pv[4], xv[4];
        lds_ld4(sP + i * Kp + 4 * kt, pv);
        lds_ld4(sX + i * rtp + 4 * rtt, xv);
#pragma unroll
        for (int kk = 0; kk < 4; kk++)
#pragma unroll
          for (int rr = 0; rr < 4; rr++) fmac_(acc[kk][rr], pv[kk], xv[rr]);
      }
    }
    __syncthreads();
  }
  // group reduction, one k row of the tiles at a time: sR[(g T + u) 4 + rr]
  cx<R>* sR = sP;
#pragma unroll
  for (int kk = 0; kk < 4; kk++) {
    if (active) {
#pragma unroll
      for (int rr = 0; rr < 4; rr++) sR[tid * 4 + rr] = acc[kk][rr];
    }
    __syncthreads();
    for (int o = tid; o < T * 4; o += kTransferTB) {
      const int uo = o >> 2, rr = o & 3;
      const int k = 4 * (uo / ntr) + kk, r = 4 * (uo % ntr) + rr;
      if (k < K && r < rt) {
        cx<R> s = sR[o];
        for (int g2 = 1; g2 < G; g2++) s = s + sR[g2 * T * 4 + o];
        P::st(yc, ((int64_t)(chi * K + k) * Vc + a) * nrhs + r0 + r, s);
      }
    }
    __syncthreads();
  }
}

// y = P x_c (mode 0), x - P x_c (mode 1), y + P x_c (mode 2), or
// xs * x + P x_c (mode 3, x stored as PX, scaled per rhs by xs and in column
// groups of xgs right-hand sides)
// P rows of a chunk sit transposed in LDS; thread u = (q, r/4) owns rows
// q, q + Q, ..., q + (TI-1) Q of the chunk (Q = rc / TI) by four right-hand
// sides, and loads the destination entries it updates before its products.
template <class P, class PM, int TI, class PX = P>
__global__ __launch_bounds__(256) void k_prolong(const typename P::S* __restrict__ xc, const typename P::S* __restrict__ x,
                                                 typename P::S* __restrict__ y, const typename PM::S* __restrict__ Pm,
                                                 TGeom t, int nrhs, int mode, int rc, int rtile,
                                                 const typename PX::S* __restrict__ xq, const double* __restrict__ xs,
                                                 int xgs) {
  using R = typename P::R;
  extern __shared__ __align__(16) char smem[];
  const int64_t a = blockIdx.x >> 1;
  const int chi = blockIdx.x & 1;
  const int r0 = blockIdx.y * rtile;
  const int rt = nrhs - r0 < rtile ? nrhs - r0 : rtile;
  const int K = t.ntv, half = t.half, rows = t.rows;
  const int rtp = round4(rt), ntr = rtp >> 2;
  const int Q = rc / TI, NT = Q * ntr;
  const int64_t Vc = t.c.V, Vf = t.f.V;
  const int tid = threadIdx.x;
  int64_t* sS = reinterpret_cast<int64_t*>(smem);                        // [bvol] fine sites
  cx<R>* sC = reinterpret_cast<cx<R>*>(smem + sites_bytes(t.bvol));      // [K][rtp] coarse values
  cx<R>* sPT = sC + (size_t)K * rtp;                                      // [K][rc] P^T of the chunk
  aggregate_sites(t, a, sS);
  for (int i = tid; i < K * rtp; i += kTransferTB) {
    const int k = i / rtp, r = i - k * rtp;
    cx<R> v = {0, 0};
    if (r < rt) v = P::ld(xc, ((int64_t)(chi * K + k) * Vc + a) * nrhs + r0 + r);
    sC[i] = v;
  }
  const typename PM::S* pb = Pm + ((a * 2 + chi) * rows) * (int64_t)K;
  const typename P::S* src = mode == 1 ? x : y;
  for (int row0 = 0; row0 < rows; row0 += rc) {
    const int nr = rows - row0 < rc ? rows - row0 : rc;
    __syncthreads();  // previous chunk consumed (and sC, sS written on the first pass)
    stage_p_rows<PM, R, true>(pb, row0, nr, K, rc, sPT);
    __syncthreads();
    for (int uo = tid; uo < NT; uo += kTransferTB) {
      const int q = uo / ntr, rtt = uo - q * ntr;
      if (q >= nr) continue;
      int64_t base[TI], frow[TI];
      cx<R> acc[TI][4];
#pragma unroll
      for (int i = 0; i < TI; i++) {
        const int ii = q + Q * i;
        base[i] = -1;
        frow[i] = 0;
        if (ii < nr) {
          const int row = row0 + ii, loc = row / half, j = row - loc * half;
          frow[i] = (int64_t)(chi * half + j) * Vf + sS[loc];
          base[i] = frow[i] * nrhs + r0 + 4 * rtt;
        }
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
          acc[i][rr] = {0, 0};
          if (mode != 0 && base[i] >= 0 && 4 * rtt + rr < rt) {
            if (mode == 3) {
              const cx<typename PX::R> u =
                  PX::ld(xq, grouped_index(frow[i], r0 + 4 * rtt + rr, nrhs, xgs, 2 * half * Vf));
              acc[i][rr] = (R)xs[r0 + 4 * rtt + rr] * cx<R>{(R)u.re, (R)u.im};
            } else {
              acc[i][rr] = P::ld(src, base[i] + rr);
            }
          }
        }
      }
      if (mode == 1) {
#pragma unroll
        for (int i = 0; i < TI; i++)
#pragma unroll
          for (int rr = 0; rr < 4; rr++) acc[i][rr] = {-acc[i][rr].re, -acc[i][rr].im};
      }
      // acc holds -x (mode 1), y (mode 2) or 0; the sum over k is added on
      // top and the sign restored for mode 1
      for (int k = 0; k < K; k++) {
        cx<R> cv[4], pv[TI];
        lds_ld4(sC + k * rtp + 4 * rtt, cv);
#pragma unroll
        for (int i = 0; i < TI; i++) pv[i] = sPT[k * rc + q + Q * i];
#pragma unroll
        for (int i = 0; i < TI; i++)
#pragma unroll
          for (int rr = 0; rr < 4; rr++) fma_(acc[i][rr], pv[i], cv[rr]);
      }
#pragma unroll
      for (int i = 0; i < TI; i++) {
        if (base[i] < 0) continue;
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
          if (4 * rtt + rr < rt) {
            cx<R> v = acc[i][rr];
            if (mode == 1) v = {-v.re, -v.im};
            P::st(y, base[i] + rr, v);
          }
        }
      }
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
  MGM_CHECK(t.ntv <= 128 && t.bvol <= 1024, MGM_ERR_SHAPE,
            "transfers support at most 128 test vectors and 1024 sites per aggregate");
  const int tile = restrict_rt(t), rt = nrhs < tile ? nrhs : tile;
  const dim3 nb((unsigned)(2 * t.c.V), (unsigned)((nrhs + tile - 1) / tile)), tb(kTransferTB);
  if (p == MGM_PREC_F64) {
    const int rc = restrict_chunk_rows(t, rt, 16);
    hipLaunchKernelGGL((k_restrict<F64, F64>), nb, tb, restrict_lds(t, rt, rc, 16), ctx->stream,
                       (const double2*)x, (double2*)yc, P64, t, nrhs, rc, tile, nullptr, nrhs);
  } else if (p == MGM_PREC_F32) {
    const int rc = restrict_chunk_rows(t, rt, 8);
    hipLaunchKernelGGL((k_restrict<F32, F16>), nb, tb, restrict_lds(t, rt, rc, 8), ctx->stream,
                       (const float2*)x, (float2*)yc, P16, t, nrhs, rc, tile, nullptr, nrhs);
  } else {
    throw Error(MGM_ERR_INVALID_ARG, "restrict: precision must be F64 or F32");
  }
  MGM_LAUNCH_CHECK();
}

void Transfer::prolong(mgm_prec p, const void* xc, const void* x, void* y, int nrhs, int mode) const {
  ProfScope ps(ctx, KC_TRANSFER, bytes(p, nrhs));
  MGM_CHECK(t.ntv <= 128 && t.bvol <= 1024, MGM_ERR_SHAPE,
            "transfers support at most 128 test vectors and 1024 sites per aggregate");
  if (p == MGM_PREC_F64) {
    const int tile = prolong_rt(t, 16), rt = nrhs < tile ? nrhs : tile;
    const dim3 nb((unsigned)(2 * t.c.V), (unsigned)((nrhs + tile - 1) / tile)), tb(kTransferTB);
    const int rc = prolong_chunk_rows(t, rt, 16, 1);
    hipLaunchKernelGGL((k_prolong<F64, F64, 1>), nb, tb, prolong_lds(t, rt, rc, 16), ctx->stream,
                       (const double2*)xc, (const double2*)x, (double2*)y, P64, t, nrhs, mode, rc, tile, nullptr,
                       nullptr, nrhs);
  } else if (p == MGM_PREC_F32) {
    const int tile = prolong_rt(t, 8), rt = nrhs < tile ? nrhs : tile;
    const dim3 nb((unsigned)(2 * t.c.V), (unsigned)((nrhs + tile - 1) / tile)), tb(kTransferTB);
    const int rc = prolong_chunk_rows(t, rt, 8, 2);
    hipLaunchKernelGGL((k_prolong<F32, F16, 2>), nb, tb, prolong_lds(t, rt, rc, 8), ctx->stream,
                       (const float2*)xc, (const float2*)x, (float2*)y, P16, t, nrhs, mode, rc, tile, nullptr,
                       nullptr, nrhs);
  } else {
    throw Error(MGM_ERR_INVALID_ARG, "prolong: precision must be F64 or F32");
  }
  MGM_LAUNCH_CHECK();
}

void Transfer::restrict16(const __half2* x16, const double* xs, float2* yc, int nrhs, int xgs) const {
  ProfScope ps(ctx, KC_TRANSFER, bytes(MGM_PREC_F32, nrhs));
  MGM_CHECK(t.ntv <= 128 && t.bvol <= 1024, MGM_ERR_SHAPE,
            "transfers support at most 128 test vectors and 1024 sites per aggregate");
  MGM_CHECK(P16 != nullptr && xs != nullptr, MGM_ERR_INVALID_ARG, "FP16 transfer input needs P16 and scales");
  if (xgs <= 0) xgs = nrhs;
  MGM_CHECK(nrhs % xgs == 0, MGM_ERR_INVALID_ARG, "column groups must divide the rhs count");
  const int tile = restrict_rt(t), rt = nrhs < tile ? nrhs : tile;
  const dim3 nb((unsigned)(2 * t.c.V), (unsigned)((nrhs + tile - 1) / tile)), tb(kTransferTB);
  const int rc = restrict_chunk_rows(t, rt, 8);
  hipLaunchKernelGGL((k_restrict<F32, F16, F16>), nb, tb, restrict_lds(t, rt, rc, 8), ctx->stream, x16, yc, P16, t,
                     nrhs, rc, tile, xs, xgs);
  MGM_LAUNCH_CHECK();
}

void Transfer::prolong16(const float2* xc, const __half2* x16, const double* xs, float2* y, int nrhs,
                         int xgs) const {
  ProfScope ps(ctx, KC_TRANSFER, bytes(MGM_PREC_F32, nrhs));
  const int tile = prolong_rt(t, 8), rt = nrhs < tile ? nrhs : tile;
  const dim3 nb((unsigned)(2 * t.c.V), (unsigned)((nrhs + tile - 1) / tile)), tb(kTransferTB);
  MGM_CHECK(t.ntv <= 128 && t.bvol <= 1024, MGM_ERR_SHAPE,
            "transfers support at most 128 test vectors and 1024 sites per aggregate");
  MGM_CHECK(P16 != nullptr && xs != nullptr, MGM_ERR_INVALID_ARG, "FP16 transfer input needs P16 and scales");
  if (xgs <= 0) xgs = nrhs;
  MGM_CHECK(nrhs % xgs == 0, MGM_ERR_INVALID_ARG, "column groups must divide the rhs count");
  const int rc = prolong_chunk_rows(t, rt, 8, 2);
  hipLaunchKernelGGL((k_prolong<F32, F16, 2, F16>), nb, tb, prolong_lds(t, rt, rc, 8), ctx->stream, xc,
                     (const float2*)nullptr, y, P16, t, nrhs, 3, rc, tile, x16, xs, xgs);
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

constexpr int kGalPairs = 16;  // (i, j) pairs per thread: d * jc <= 256 * kGalPairs

// Both Galerkin kernels run one workgroup per (coarse site, stencil
// direction, chunk of jc coarse columns j).  For every fine site x of the
// aggregate, the sum over the hops k of x that land in that direction of
// B[x, k] P(y_k) (the chunk's columns) is staged in LDS, and each thread
// accumulates up to kGalPairs entries (i, j) of P(x)^H times that sum.
__global__ void k_galerkin_fine(FineOp op, TGeom t, const double2* __restrict__ Pm, double2* __restrict__ Ac,
                                int jc) {
  extern __shared__ double2 T[];  // [12][jc] hop sums, then [2][6][ntv] rows of P(x)
  const int64_t a = blockIdx.x;
  const int tgt = blockIdx.y;
  const int j0 = blockIdx.z * jc;
  const int d = 2 * t.ntv, ntv = t.ntv, tid = threadIdx.x;
  const int nj = d - j0 < jc ? d - j0 : jc;
  double2* PX = T + 12 * jc;
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
    bool any = false;
    for (int k = 0; k < 9; k++) any |= hop_target(k, l, t.b) == tgt;
    if (!any) continue;  // uniform over the workgroup
    for (int m = 0; m < 4; m++) fc[m] = ca[m] * t.b[m] + l[m];
    const int64_t s = index_of(t.f, fc);
    if (tid < nj) {
      const int j = j0 + tid, chij = j / ntv, kk = j % ntv;
      cx<double> sum[12];
      for (int m = 0; m < 12; m++) sum[m] = {0, 0};
      for (int k = 0; k < 9; k++) {
        if (hop_target(k, l, t.b) != tgt) continue;
        const int64_t y = hop_neighbour(t.f, fc, k);
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
        for (int m = 0; m < 12; m++) sum[m] = sum[m] + o[m];
      }
      for (int m = 0; m < 12; m++) T[m * jc + tid] = make_double2(sum[m].re, sum[m].im);
    }
    for (int e = tid; e < 12 * ntv; e += blockDim.x) {
      const int chi = e / (6 * ntv), r = e - chi * 6 * ntv;  // r = m ntv + k
      PX[e] = Pm[((a * 2 + chi) * t.rows + loc * 6) * (int64_t)ntv + r];
    }
    __syncthreads();
    for (int q = 0; q < kGalPairs; q++) {
      int pidx = tid + q * blockDim.x;
      if (pidx >= d * nj) break;
      int i = pidx / nj, jj = pidx % nj;
      int chii = i / ntv, ki = i % ntv;
      const double2* pr = PX + chii * 6 * ntv + ki;
      for (int m = 0; m < 6; m++) {
        double2 pv = pr[m * ntv];
        double2 tv = T[(6 * chii + m) * jc + jj];
        fmac_(acc[q], cx<double>{pv.x, pv.y}, cx<double>{tv.x, tv.y});
      }
    }
    __syncthreads();
  }
  const int64_t Vc = t.c.V;
  for (int q = 0; q < kGalPairs; q++) {
    int pidx = tid + q * blockDim.x;
    if (pidx >= d * nj) break;
    int i = pidx / nj, j = j0 + pidx % nj;
    Ac[((int64_t)(tgt * d + i) * d + j) * Vc + a] = make_double2(acc[q].re, acc[q].im);
  }
}

__global__ void k_galerkin_coarse(CoarseOp op, TGeom t, const double2* __restrict__ Pm, double2* __restrict__ Ac,
                                  int jc) {
  extern __shared__ double2 T[];  // [dl][jc]
  const int64_t a = blockIdx.x;
  const int tgt = blockIdx.y;
  const int j0 = blockIdx.z * jc;
  const int d = 2 * t.ntv, ntv = t.ntv, tid = threadIdx.x;
  const int nj = d - j0 < jc ? d - j0 : jc;
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
    bool any = false;
    for (int k = 0; k < 9; k++) any |= hop_target(k, l, t.b) == tgt;
    if (!any) continue;  // uniform over the workgroup
    for (int m = 0; m < 4; m++) fc[m] = ca[m] * t.b[m] + l[m];
    const int64_t s = index_of(t.f, fc);
    // entries (i2, jj) of the chunk's hop sum, one per thread at a time
    for (int e = tid; e < dl * nj; e += blockDim.x) {
      const int i2 = e / nj, jj = e - i2 * nj;
      const int j = j0 + jj, chij = j / ntv, kk = j % ntv;
      cx<double> o = {0, 0};
      for (int k = 0; k < 9; k++) {
        if (hop_target(k, l, t.b) != tgt) continue;
        const int64_t y = hop_neighbour(t.f, fc, k);
        int64_t ay;
        int locy;
        agg_of(t, y, ay, locy);
        const double2* py = Pm + ((ay * 2 + chij) * t.rows + locy * hl) * (int64_t)ntv + kk;
        const double2* Arow = op.A64 + ((int64_t)(k * dl + i2) * dl + chij * hl) * Vl + s;
        for (int mm = 0; mm < hl; mm++) {
          double2 av = Arow[(int64_t)mm * Vl];
          double2 pv = py[(int64_t)mm * ntv];
          fma_(o, cx<double>{av.x, av.y}, cx<double>{pv.x, pv.y});
        }
      }
      T[i2 * jc + jj] = make_double2(o.re, o.im);
    }
    __syncthreads();
    for (int q = 0; q < kGalPairs; q++) {
      int pidx = tid + q * blockDim.x;
      if (pidx >= d * nj) break;
      int i = pidx / nj, jj = pidx % nj;
      int chii = i / ntv, ki = i % ntv;
      const double2* pr = Pm + ((a * 2 + chii) * t.rows + loc * hl) * (int64_t)ntv + ki;
      for (int mm = 0; mm < hl; mm++) {
        double2 pv = pr[(int64_t)mm * ntv];
        double2 tv = T[(chii * hl + mm) * jc + jj];
        fmac_(acc[q], cx<double>{pv.x, pv.y}, cx<double>{tv.x, tv.y});
      }
    }
    __syncthreads();
  }
  const int64_t Vc = t.c.V;
  for (int q = 0; q < kGalPairs; q++) {
    int pidx = tid + q * blockDim.x;
    if (pidx >= d * nj) break;
    int i = pidx / nj, j = j0 + pidx % nj;
    Ac[((int64_t)(tgt * d + i) * d + j) * Vc + a] = make_double2(acc[q].re, acc[q].im);
  }
}

// columns per Galerkin workgroup: all d when the pairs and the staged rows
// fit, else the largest power of two that does
static int galerkin_jc(int d, int rows_staged) {
  int jc = d;
  while (jc > 1 && ((size_t)d * jc > (size_t)256 * kGalPairs || (size_t)rows_staged * jc * sizeof(double2) > 65536))
    jc = (jc + 1) / 2;
  return jc;
}

void mg_galerkin_fine(Context* c, const FineOp& op, const Transfer& T, CoarseOp& out) {
  const TGeom& t = T.t;
  const int d = 2 * t.ntv;
  MGM_CHECK(d <= 256, MGM_ERR_SHAPE, "too many test vectors");
  const int jc = galerkin_jc(d, 12);
  const size_t sh = (size_t)12 * (jc + t.ntv) * sizeof(double2);
  hipLaunchKernelGGL(k_galerkin_fine, dim3((unsigned)t.c.V, 9, (unsigned)((d + jc - 1) / jc)), dim3(256), sh,
                     c->stream, op, t, T.P64, out.A64, jc);
  MGM_LAUNCH_CHECK();
}

void mg_galerkin_coarse(Context* c, const CoarseOp& op, const Transfer& T, CoarseOp& out) {
  const TGeom& t = T.t;
  const int d = 2 * t.ntv;
  MGM_CHECK(d <= 256 && t.f.dof <= 256, MGM_ERR_SHAPE, "too many test vectors");
  const int jc = galerkin_jc(d, t.f.dof);
  const size_t sh = (size_t)t.f.dof * jc * sizeof(double2);
  hipLaunchKernelGGL(k_galerkin_coarse, dim3((unsigned)t.c.V, 9, (unsigned)((d + jc - 1) / jc)), dim3(256), sh,
                     c->stream, op, t, T.P64, out.A64, jc);
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
