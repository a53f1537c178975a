// Coarse stencil y(s) = sum_dir A_dir(s) x(nbr(s, dir)) on the matrix cores.
//
// Per coarse site the nine d x d complex blocks multiply d x nrhs neighbour
// blocks: a dense contraction over (dir, j), done by one wave per
// (site, 16 right-hand sides).  A is read once, from a fragment-packed copy
// in which every MFMA A-operand of a wave is one contiguous 1 KB chunk; the
// neighbour block is the B operand.  Complex products use real MFMAs:
//   Re y += Re A Re x - Im A Im x,   Im y += Re A Im x + Im A Re x.
// FP64 / FP32: v_mfma_{f64,f32}_16x16x4 (A[i][k]: lane = i%16 + 16 k;
// B[k][n]: lane = n + 16 k; D[i][n]: lane = n + 16 q with row i = 4 q + reg
// for FP32 and i = q + 4 reg for FP64 -- checked on the device).
// BF16 (mixed form): v_mfma_f32_16x16x16 bf16 with FP32 accumulation
// (A: lane holds k = 4 (lane/16) .. +3 of row lane%16; B likewise by column).
// BF16 values are rounded to nearest even from FP32.
#include "mg.h"

namespace mgm {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void coords_c(const LGeom& g, int64_t s, int c[4]) {
  c[0] = (int)(s % g.dims[0]); s /= g.dims[0];
  c[1] = (int)(s % g.dims[1]); s /= g.dims[1];
  c[2] = (int)(s % g.dims[2]); s /= g.dims[2];
  c[3] = (int)s;
}
__device__ __forceinline__ int64_t nbr_c(const LGeom& g, const int c[4], int dir) {
  int cc[4] = {c[0], c[1], c[2], c[3]};
  if (dir > 0) {
    int mu = (dir - 1) & 3;
    cc[mu] += (dir <= 4) ? 1 : -1;
    cc[mu] = (cc[mu] + g.dims[mu]) % g.dims[mu];
  }
  return cc[0] + (int64_t)g.dims[0] * (cc[1] + (int64_t)g.dims[1] * (cc[2] + (int64_t)g.dims[2] * cc[3]));
}

struct MGeo {
  int d, MT, KC64, KC16;
};
static MGeo mgeo(int d) {
  MGeo m;
  m.d = d;
  m.MT = (d + 15) / 16;
  m.KC64 = (d + 3) / 4;
  m.KC16 = (d + 15) / 16;
  return m;
}

size_t mg_mfma_bytes(const CoarseOp& A) {
  MGeo m = mgeo(A.d);
  return (size_t)A.g.V * 9 * m.KC16 * m.MT * 2 * 64 * 4 * sizeof(uint16_t);
}
size_t mg_mfma64_bytes(const CoarseOp& A) {
  MGeo m = mgeo(A.d);
  return (size_t)A.g.V * 9 * m.KC64 * m.MT * 64 * sizeof(double2);
}

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// ---------------------------------------------------------------- packing

__global__ void k_pack64(double2* __restrict__ out, const double2* __restrict__ A, LGeom g, MGeo m) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)9 * m.KC64 * m.MT * 64;
  if (e >= g.V * per) return;
  const int64_t s = e / per;
  int64_t q = e % per;
  const int lane = (int)(q % 64); q /= 64;
  const int mt = (int)(q % m.MT); q /= m.MT;
  const int kc = (int)(q % m.KC64);
  const int dir = (int)(q / m.KC64);
  const int i = 16 * mt + (lane & 15), k = 4 * kc + (lane >> 4);
  double2 v = make_double2(0, 0);
  if (i < m.d && k < m.d) v = A[((int64_t)(dir * m.d + i) * m.d + k) * g.V + s];
  out[e] = v;
}

__global__ void k_pack_bf16(uint16_t* __restrict__ out, const double2* __restrict__ A, LGeom g, MGeo m) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)9 * m.KC16 * m.MT * 2 * 64 * 4;
  if (e >= g.V * per) return;
  const int64_t s = e / per;
  int64_t q = e % per;
  const int el = (int)(q % 4); q /= 4;
  const int lane = (int)(q % 64); q /= 64;
  const int part = (int)(q % 2); q /= 2;  // 0: real, 1: imaginary
  const int mt = (int)(q % m.MT); q /= m.MT;
  const int kc = (int)(q % m.KC16);
  const int dir = (int)(q / m.KC16);
  const int i = 16 * mt + (lane & 15), k = 16 * kc + 4 * (lane >> 4) + el;
  float v = 0.0f;
  if (i < m.d && k < m.d) {
    double2 a = A[((int64_t)(dir * m.d + i) * m.d + k) * g.V + s];
    v = (float)(part ? a.y : a.x);
  }
  out[e] = bf16_rne(v);
}

void mg_mfma_pack(Context* c, CoarseOp& A) {
  MGeo m = mgeo(A.d);
  if (A.Abf) {
    int64_t n = A.g.V * 9 * m.KC16 * m.MT * 2 * 64 * 4;
    hipLaunchKernelGGL(k_pack_bf16, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, (uint16_t*)A.Abf, A.A64,
                       A.g, m);
    MGM_LAUNCH_CHECK();
  }
}

void mg_mfma64_pack(Context* c, CoarseOp& A) {
  MGeo m = mgeo(A.d);
  int64_t n = A.g.V * 9 * m.KC64 * m.MT * 64;
  hipLaunchKernelGGL(k_pack64, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, A.Ap64, A.A64, A.g, m);
  MGM_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- apply

// 16x16x4 MFMA in FP64 or FP32 (same lane layout, one A and one B value per lane)
// Output row of accumulator register j in lane group q = lane/16 (column
// lane%16): FP64 interleaves rows (4 j + q), FP32 keeps them blocked (4 q + j).
struct M64 {
  using R = double;
  using C2 = double2;
  using V4 = d4_t;
  __device__ static V4 mfma(R a, R b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int q, int j) { return 4 * j + q; }
};
struct M32 {
  using R = float;
  using C2 = float2;
  using V4 = f4_t;
  __device__ static V4 mfma(R a, R b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int q, int j) { return 4 * q + j; }
};

template <class M, int MT, int MAXT = 256>
__global__ __launch_bounds__(MAXT) void k_coarse_mfma4(const typename M::C2* __restrict__ x,
                                                     typename M::C2* __restrict__ y,
                                                     const typename M::C2* __restrict__ Ap, LGeom g, int d, int KC,
                                                     int nrhs, int ntr, int wpb) {
  using R = typename M::R;
  using V4 = typename M::V4;
  using C2 = typename M::C2;
  // one workgroup per site and group of wpb 16-rhs tiles (one wave each):
  // the tiles of a site stream the same A fragments through the CU's caches
  // at the same time
  const int64_t s = blockIdx.x;
  const int nt = blockIdx.y * wpb + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (nt >= ntr) return;
  const int n = lane & 15, kq = lane >> 4;
  const int r = nt * 16 + n;
  const int64_t V = g.V;
  int c[4];
  coords_c(g, s, c);
  V4 yr[MT], yi[MT];
#pragma unroll
  for (int mt = 0; mt < MT; mt++) {
    yr[mt] = (V4){0, 0, 0, 0};
    yi[mt] = (V4){0, 0, 0, 0};
  }
  const C2* As = Ap + (int64_t)s * 9 * KC * MT * 64 + lane;
#pragma unroll 1
  for (int dir = 0; dir < 9; dir++) {
    const int64_t sn = nbr_c(g, c, dir);
    const C2* Ad = As + (int64_t)dir * KC * MT * 64;
#pragma unroll 4
    for (int kc = 0; kc < KC; kc++) {
      const int k = 4 * kc + kq;
      C2 xv = {0, 0};
      if (k < d && r < nrhs) xv = x[((int64_t)k * V + sn) * nrhs + r];
#pragma unroll
      for (int mt = 0; mt < MT; mt++) {
        const C2 a = Ad[(int64_t)(kc * MT + mt) * 64];
        yr[mt] = M::mfma(a.x, xv.x, yr[mt]);
        yr[mt] = M::mfma(-a.y, xv.y, yr[mt]);
        yi[mt] = M::mfma(a.x, xv.y, yi[mt]);
        yi[mt] = M::mfma(a.y, xv.x, yi[mt]);
      }
    }
  }
  if (r < nrhs) {
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int i = 16 * mt + M::row(kq, j);
        if (i < d) y[((int64_t)i * V + s) * nrhs + r] = C2{(R)yr[mt][j], (R)yi[mt][j]};
      }
  }
}

template <int MT, int NT, int MAXT = 256>
__global__ __launch_bounds__(MAXT) void k_coarse_mfma_bf16(const float2* __restrict__ x, float2* __restrict__ y,
                                                         const uint16_t* __restrict__ Ap, LGeom g, int d,
                                                         int nrhs, int ntr, int wpb) {
  // K chunks of 16 = ceil(d / 16) = MT: the chunk loop unrolls completely so
  // every fragment load of a direction is in flight at once
  constexpr int KC = MT;
  // one workgroup per site and group of wpb waves, each wave NT consecutive
  // 16-rhs tiles: a wave loads every A fragment once for its NT tiles, and
  // the waves of a site stream the same fragments through the CU's caches
  const int64_t s = blockIdx.x;
  const int nt0 = (blockIdx.y * wpb + (threadIdx.x >> 6)) * NT;
  const int lane = threadIdx.x & 63;
  if (nt0 >= ntr) return;
  const int n = lane & 15, kq = lane >> 4;
  const int64_t V = g.V;
  int c[4];
  coords_c(g, s, c);
  f4_t yr[NT][MT], yi[NT][MT];
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int mt = 0; mt < MT; mt++) {
      yr[t][mt] = (f4_t){0, 0, 0, 0};
      yi[t][mt] = (f4_t){0, 0, 0, 0};
    }
  const uint16_t* As = Ap + (int64_t)s * 9 * KC * MT * 512 + lane * 4;
#pragma unroll 1
  for (int dir = 0; dir < 9; dir++) {
    const int64_t sn = nbr_c(g, c, dir);
    const uint16_t* Ad = As + (int64_t)dir * KC * MT * 512;
#pragma unroll
    for (int kc = 0; kc < KC; kc++) {
      s4_t ar[MT], ai[MT], nai[MT];
#pragma unroll
      for (int mt = 0; mt < MT; mt++) {
        const uint16_t* f = Ad + (int64_t)(kc * MT + mt) * 512;
        ar[mt] = *(const s4_t*)f;
        ai[mt] = *(const s4_t*)(f + 256);
        nai[mt] = ai[mt] ^ (s4_t){(short)0x8000, (short)0x8000, (short)0x8000, (short)0x8000};
      }
#pragma unroll
      for (int t = 0; t < NT; t++) {
        const int r = (nt0 + t) * 16 + n;
        s4_t br, bi;
#pragma unroll
        for (int el = 0; el < 4; el++) {
          const int k = 16 * kc + 4 * kq + el;
          float2 xv = make_float2(0.f, 0.f);
          if (k < d && r < nrhs) xv = x[((int64_t)k * V + sn) * nrhs + r];
          br[el] = (short)bf16_rne(xv.x);
          bi[el] = (short)bf16_rne(xv.y);
        }
#pragma unroll
        for (int mt = 0; mt < MT; mt++) {
          yr[t][mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar[mt], br, yr[t][mt], 0, 0, 0);
          yr[t][mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(nai[mt], bi, yr[t][mt], 0, 0, 0);
          yi[t][mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar[mt], bi, yi[t][mt], 0, 0, 0);
          yi[t][mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai[mt], br, yi[t][mt], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; t++) {
    const int r = (nt0 + t) * 16 + n;
    if (r < nrhs) {
#pragma unroll
      for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int i = 16 * mt + 4 * kq + j;
          if (i < d) y[((int64_t)i * V + s) * nrhs + r] = make_float2(yr[t][mt][j], yi[t][mt][j]);
        }
    }
  }
}

#define MT_DISPATCH(MTV, ...)                       \
  switch (MTV) {                                    \
    case 1: { constexpr int MTc = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int MTc = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int MTc = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int MTc = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int MTc = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int MTc = 6; __VA_ARGS__; } break; \
    case 7: { constexpr int MTc = 7; __VA_ARGS__; } break; \
    case 8: { constexpr int MTc = 8; __VA_ARGS__; } break; \
    case 9: { constexpr int MTc = 9; __VA_ARGS__; } break; \
    case 10: { constexpr int MTc = 10; __VA_ARGS__; } break; \
    case 11: { constexpr int MTc = 11; __VA_ARGS__; } break; \
    case 12: { constexpr int MTc = 12; __VA_ARGS__; } break; \
    case 13: { constexpr int MTc = 13; __VA_ARGS__; } break; \
    case 14: { constexpr int MTc = 14; __VA_ARGS__; } break; \
    case 15: { constexpr int MTc = 15; __VA_ARGS__; } break; \
    case 16: { constexpr int MTc = 16; __VA_ARGS__; } break; \
    default: throw Error(MGM_ERR_SHAPE, "coarse dof must be <= 256"); \
  }

// the 512-thread shapes and two tiles per wave exist up to eight row tiles
// (their registers)
#define MT_DISPATCH8(MTV, ...)                      \
  switch (MTV) {                                    \
    case 1: { constexpr int MTc = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int MTc = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int MTc = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int MTc = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int MTc = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int MTc = 6; __VA_ARGS__; } break; \
    case 7: { constexpr int MTc = 7; __VA_ARGS__; } break; \
    case 8: { constexpr int MTc = 8; __VA_ARGS__; } break; \
    default: throw Error(MGM_ERR_INVALID_ARG, "coarse shape not built for more than eight row tiles"); \
  }

// Waves (16-rhs tiles) per workgroup of at most 256 threads: 4 by default
// (the autotuner also tries 2 and 1); v indexes the distinct candidates for
// ntr tiles.
static int wpb_of(int ntr, int v) {
  int cand[3] = {std::min(ntr, 4), std::min(ntr, 2), 1}, n = 0, out[3];
  for (int c : cand) {
    bool seen = false;
    for (int k = 0; k < n; k++) seen |= out[k] == c;
    if (!seen) out[n++] = c;
  }
  return out[v < n ? v : 0];
}
static int wpb_count(int ntr) { return ntr >= 4 ? 3 : ntr >= 2 ? 2 : 1; }
// FP64 / FP32 shapes: the wpb_of candidates, then (5 to 8 tiles) every tile
// of a site in one workgroup of up to 512 threads, so that the site's A
// fragments are read from HBM once and shared through the CU's cache
static int shapes4_count(int ntr, int mt) { return wpb_count(ntr) + (ntr > 4 && ntr <= 8 && mt <= 8 ? 1 : 0); }
static int wpb4_of(int ntr, int v) { return v < wpb_count(ntr) ? wpb_of(ntr, v) : ntr; }

void coarse_apply_mfma64(const CoarseOp& A, const double2* x, double2* y, int nrhs) {
  MGeo m = mgeo(A.d);
  const int ntr = (nrhs + 15) / 16;
  ProfScope ps(A.ctx, KC_COARSE_F64, A.bytes(MGM_PREC_F64, nrhs));
  A.ctx->choose("coarse64/" + std::to_string(A.g.V) + "/" + std::to_string(A.d) + "/" + std::to_string(nrhs),
                shapes4_count(ntr, m.MT), [&](int v) {
                  MGM_CHECK(v >= 0 && v < shapes4_count(ntr, m.MT), MGM_ERR_INVALID_ARG,
                            "coarse launch variant out of range");
                  const int wpb = wpb4_of(ntr, v);
                  const dim3 nb((unsigned)A.g.V, (unsigned)((ntr + wpb - 1) / wpb)), tb(64 * wpb);
                  if (wpb > 4) {
                    MT_DISPATCH8(m.MT, hipLaunchKernelGGL((k_coarse_mfma4<M64, MTc, 512>), nb, tb, 0, A.ctx->stream,
                                                         x, y, A.Ap64, A.g, A.d, m.KC64, nrhs, ntr, wpb));
                  } else {
                    MT_DISPATCH(m.MT, hipLaunchKernelGGL((k_coarse_mfma4<M64, MTc>), nb, tb, 0, A.ctx->stream, x,
                                                         y, A.Ap64, A.g, A.d, m.KC64, nrhs, ntr, wpb));
                  }
                  MGM_LAUNCH_CHECK();
                });
}

void coarse_apply_mfma32(const CoarseOp& A, const float2* x, float2* y, int nrhs) {
  MGeo m = mgeo(A.d);
  const int ntr = (nrhs + 15) / 16;
  ProfScope ps(A.ctx, KC_COARSE_F32, A.bytes(MGM_PREC_F32, nrhs));
  A.ctx->choose("coarse32/" + std::to_string(A.g.V) + "/" + std::to_string(A.d) + "/" + std::to_string(nrhs),
                shapes4_count(ntr, m.MT), [&](int v) {
                  MGM_CHECK(v >= 0 && v < shapes4_count(ntr, m.MT), MGM_ERR_INVALID_ARG,
                            "coarse launch variant out of range");
                  const int wpb = wpb4_of(ntr, v);
                  const dim3 nb((unsigned)A.g.V, (unsigned)((ntr + wpb - 1) / wpb)), tb(64 * wpb);
                  if (wpb > 4) {
                    MT_DISPATCH8(m.MT, hipLaunchKernelGGL((k_coarse_mfma4<M32, MTc, 512>), nb, tb, 0, A.ctx->stream,
                                                         x, y, A.A32, A.g, A.d, m.KC64, nrhs, ntr, wpb));
                  } else {
                    MT_DISPATCH(m.MT, hipLaunchKernelGGL((k_coarse_mfma4<M32, MTc>), nb, tb, 0, A.ctx->stream, x,
                                                         y, A.A32, A.g, A.d, m.KC64, nrhs, ntr, wpb));
                  }
                  MGM_LAUNCH_CHECK();
                });
}

__global__ void k_pack32(float2* __restrict__ out, const double2* __restrict__ packed64, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = make_float2((float)packed64[e].x, (float)packed64[e].y);
}

size_t mg_mfma32_bytes(const CoarseOp& A) { return mg_mfma64_bytes(A) / 2; }

void mg_mfma32_pack(Context* c, CoarseOp& A) {
  MGeo m = mgeo(A.d);
  int64_t n = A.g.V * 9 * m.KC64 * m.MT * 64;
  hipLaunchKernelGGL(k_pack32, dim3(nblocks_for(n, 256)), dim3(256), 0, c->stream, A.A32, A.Ap64, n);
  MGM_LAUNCH_CHECK();
}

void coarse_apply_mfma(const CoarseOp& A, const float2* x, float2* y, int nrhs) {
  MGM_CHECK(A.Abf != nullptr, MGM_ERR_INVALID_ARG, "BF16 coarse stencil not built (mixed == 0)");
  MGeo m = mgeo(A.d);
  const int ntr = (nrhs + 15) / 16;
  ProfScope ps(A.ctx, KC_COARSE_BF16, A.bytes(MGM_PREC_BF16, nrhs));
  // shapes: one tile per wave with 4 / 2 / 1 waves per workgroup, then two
  // and four tiles per wave (fewer A fragment loads per rhs); with more than
  // four tiles, also every tile of a site in one workgroup of up to 8 waves
  // (one or two tiles per wave), so that the site's A fragments are read
  // from HBM once and shared through the CU's cache
  struct Shape {
    int wpb, nt;
  };
  std::vector<Shape> shapes;
  for (int v = 0; v < wpb_count(ntr); v++) shapes.push_back({wpb_of(ntr, v), 1});
  if (ntr >= 2 && m.MT <= 8) shapes.push_back({1, 2});
  if (ntr >= 4 && m.MT <= 8) shapes.push_back({2, 2});
  if (ntr >= 4 && m.MT <= 3) shapes.push_back({1, 4});
  if (ntr >= 8 && m.MT <= 3) shapes.push_back({2, 4});
  const size_t n_small = shapes.size();
  if (ntr > 4 && ntr <= 8 && m.MT <= 8) shapes.push_back({ntr, 1});
  if (ntr > 4 && ntr <= 16 && m.MT <= 4) shapes.push_back({(ntr + 1) / 2, 2});
  A.ctx->choose("coarsebf16/" + std::to_string(A.g.V) + "/" + std::to_string(A.d) + "/" + std::to_string(nrhs),
                (int)shapes.size(), [&](int v) {
                  MGM_CHECK(v >= 0 && v < (int)shapes.size(), MGM_ERR_INVALID_ARG,
                            "coarse launch variant out of range");
                  const int wpb = shapes[v].wpb, tpw = shapes[v].nt;
                  const int groups = (ntr + tpw - 1) / tpw;
                  const dim3 nb((unsigned)A.g.V, (unsigned)((groups + wpb - 1) / wpb)), tb(64 * wpb);
                  if ((size_t)v >= n_small) {
                    // workgroups of up to 512 threads
                    if (tpw == 1) {
                      MT_DISPATCH8(m.MT, hipLaunchKernelGGL((k_coarse_mfma_bf16<MTc, 1, 512>), nb, tb, 0,
                                                           A.ctx->stream, x, y, (const uint16_t*)A.Abf, A.g, A.d,
                                                           nrhs, ntr, wpb));
                    } else {
                      switch (m.MT) {
                        case 1: hipLaunchKernelGGL((k_coarse_mfma_bf16<1, 2, 512>), nb, tb, 0, A.ctx->stream, x, y,
                                                   (const uint16_t*)A.Abf, A.g, A.d, nrhs, ntr, wpb); break;
                        case 2: hipLaunchKernelGGL((k_coarse_mfma_bf16<2, 2, 512>), nb, tb, 0, A.ctx->stream, x, y,
                                                   (const uint16_t*)A.Abf, A.g, A.d, nrhs, ntr, wpb); break;
                        case 3: hipLaunchKernelGGL((k_coarse_mfma_bf16<3, 2, 512>), nb, tb, 0, A.ctx->stream, x, y,
                                                   (const uint16_t*)A.Abf, A.g, A.d, nrhs, ntr, wpb); break;
                        default: hipLaunchKernelGGL((k_coarse_mfma_bf16<4, 2, 512>), nb, tb, 0, A.ctx->stream, x,
                                                    y, (const uint16_t*)A.Abf, A.g, A.d, nrhs, ntr, wpb); break;
                      }
                    }
                  } else if (tpw == 1) {
                    MT_DISPATCH(m.MT, hipLaunchKernelGGL((k_coarse_mfma_bf16<MTc, 1>), nb, tb, 0, A.ctx->stream, x,
                                                         y, (const uint16_t*)A.Abf, A.g, A.d, nrhs, ntr, wpb));
                  } else if (tpw == 2) {
                    MT_DISPATCH8(m.MT, hipLaunchKernelGGL((k_coarse_mfma_bf16<MTc, 2>), nb, tb, 0, A.ctx->stream, x,
                                                         y, (const uint16_t*)A.Abf, A.g, A.d, nrhs, ntr, wpb));
                  } else {
                    switch (m.MT) {
                      case 1: hipLaunchKernelGGL((k_coarse_mfma_bf16<1, 4>), nb, tb, 0, A.ctx->stream, x, y,
                                                 (const uint16_t*)A.Abf, A.g, A.d, nrhs, ntr, wpb); break;
                      case 2: hipLaunchKernelGGL((k_coarse_mfma_bf16<2, 4>), nb, tb, 0, A.ctx->stream, x, y,
                                                 (const uint16_t*)A.Abf, A.g, A.d, nrhs, ntr, wpb); break;
                      default: hipLaunchKernelGGL((k_coarse_mfma_bf16<3, 4>), nb, tb, 0, A.ctx->stream, x, y,
                                                  (const uint16_t*)A.Abf, A.g, A.d, nrhs, ntr, wpb); break;
                    }
                  }
                  MGM_LAUNCH_CHECK();
                });
}

}  // namespace mgm
