// Probe vectors (Sec. 1: Z4, eq. z4, and the Z2, U(1) and Gaussian
// distributions named after eq. variance-Frobenius-Relation) from the
// counter-based Philox4x32-10
// generator (Salmon, Moraes, Dror, Shaw, SC'11): every entry is an
// independent function of (seed, stream, probe, index), so any probe range can
// be drawn in any batch and reproduced bit for bit.
#include "probe.h"
#include "devonce.h"

namespace mgm {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k.x += W0;
      k.y += W1;
    }
    uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

// element e = (dof * nsite + site) * nprobe + rhs, entry index i = site*dof + dof.
// slice >= 0 keeps only sites of that time slice (sites_per_slice consecutive
// sites per slice), colour >= 0 only sites of that colour of the p^4 block
// pattern (x mod p) + p((y mod p) + p((z mod p) + p(t mod p))); others are zero.
// Distributions from the Philox words w: Z4 (1, i, -1, -i)[w0 >> 30]; Z2
// 1 - 2 (w0 >> 31); U(1) exp(2 pi i (w0 + 1/2) 2^-32); real N(0, 1) by Box and
// Muller (1958) from u1 = (w0 + 1) 2^-32, u2 = w1 2^-32.
template <class P>
__global__ void k_noise(typename P::S* out, uint2 key, uint32_t stream, uint64_t first, int nprobe, int64_t nsite,
                        int dof, int kind, NoiseMask mk) {
  using R = typename P::R;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t n = nsite * dof * nprobe;
  if (e >= n) return;
  int r = (int)(e % nprobe);
  int64_t q = e / nprobe;
  int64_t site = q % nsite;
  int d = (int)(q / nsite);
  if (mk.slice >= 0 && site / mk.sites_per_slice != mk.slice) {
    P::st(out, e, cx<R>{0, 0});
    return;
  }
  if (mk.colour >= 0) {
    const int p = mk.p;
    const int64_t x = site % mk.X, y = (site / mk.X) % mk.Y, z = (site / ((int64_t)mk.X * mk.Y)) % mk.Z,
                  t = site / ((int64_t)mk.X * mk.Y * mk.Z);
    const int64_t col = x % p + p * (y % p + p * (z % p + p * (t % p)));
    if (col != mk.colour) {
      P::st(out, e, cx<R>{0, 0});
      return;
    }
  }
  uint64_t i = (uint64_t)site * dof + d;
  uint64_t pr = first + r;
  uint4 w = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), (uint32_t)pr, stream), key);
  cx<R> v;
  if (kind == MGM_NOISE_Z2) {
    v = {(R)((w.x >> 31) ? -1 : 1), 0};
  } else if (kind == MGM_NOISE_U1) {
    const double th = 6.283185307179586476925287 * ((double)w.x + 0.5) * 0x1p-32;
    v = {(R)cos(th), (R)sin(th)};
  } else if (kind == MGM_NOISE_GAUSS) {
    const double u1 = ((double)w.x + 1.0) * 0x1p-32, u2 = (double)w.y * 0x1p-32;
    v = {(R)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925287 * u2)), 0};
  } else {
    switch (w.x >> 30) {
      case 0: v = {1, 0}; break;
      case 1: v = {0, 1}; break;
      case 2: v = {-1, 0}; break;
      default: v = {0, -1}; break;
    }
  }
  P::st(out, e, v);
}

void draw_noise(Context* c, int kind, uint64_t seed, uint32_t stream, uint64_t first, int nprobe, int64_t nsite,
                int dof, mgm_prec prec, void* out, const NoiseMask& mk) {
  MGM_CHECK(kind >= MGM_NOISE_Z4 && kind <= MGM_NOISE_GAUSS, MGM_ERR_INVALID_ARG, "unknown probe distribution");
  MGM_CHECK(mk.colour < 0 || (mk.p >= 1 && mk.X % mk.p == 0 && mk.Y % mk.p == 0 && mk.Z % mk.p == 0),
            MGM_ERR_INVALID_ARG, "probing distance must divide the lattice");
  int64_t n = nsite * dof * nprobe;
  if (n == 0) return;
  uint2 key = make_uint2((uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  unsigned nb = nblocks_for(n, 256);
  if (prec == MGM_PREC_F64)
    hipLaunchKernelGGL(k_noise<F64>, dim3(nb), dim3(256), 0, c->stream, (double2*)out, key, stream, first, nprobe,
                       nsite, dof, kind, mk);
  else if (prec == MGM_PREC_F32)
    hipLaunchKernelGGL(k_noise<F32>, dim3(nb), dim3(256), 0, c->stream, (float2*)out, key, stream, first, nprobe,
                       nsite, dof, kind, mk);
  else
    throw Error(MGM_ERR_INVALID_ARG, "probe draws: precision must be F64 or F32");
  MGM_LAUNCH_CHECK();
}

void draw_z4(Context* c, uint64_t seed, uint32_t stream, uint64_t first, int nprobe, int64_t nsite, int dof,
             mgm_prec prec, void* out, int slice, int64_t sites_per_slice) {
  NoiseMask mk;
  mk.slice = slice;
  mk.sites_per_slice = sites_per_slice;
  draw_noise(c, MGM_NOISE_Z4, seed, stream, first, nprobe, nsite, dof, prec, out, mk);
}

// ------------------------------------------------------ slice reductions

// Correlator slice pairs: out[p][rhs][t] = sum_{x in slice t} sum_dof
// conj(b_{s(p)}(x)) a_{r(p)}(x) over fine vectors (dof 12).  One block per
// (slice, chunk of the slice's sites); thread = (site lane, rhs) with a fixed
// rhs; per-block partials are summed in a second fixed-order kernel.
constexpr int kSliceChunks = 32;

// Sums sh[q + k*nrhs] over k for q < nrhs (fixed order); result in sh[q].
__device__ __forceinline__ void rhs_reduce(double2* sh, int nrhs, int tp) {
  __syncthreads();
  if ((int)threadIdx.x < nrhs) {
    double a = 0, b = 0;
    for (int k = 0; k < tp; k++) {
      a += sh[threadIdx.x + k * nrhs].x;
      b += sh[threadIdx.x + k * nrhs].y;
    }
    sh[256 + threadIdx.x] = make_double2(a, b);
  }
  __syncthreads();
}

__global__ void k_slice_pairs(SliceArgs A, int64_t Vs, int T, int nrhs, double2* partial) {
  __shared__ double2 sh[512];
  const int t = blockIdx.y;
  const int chunk = blockIdx.x;
  const int64_t N = Vs * T * nrhs;
  const int tp = 256 / nrhs;
  const int r = threadIdx.x % nrhs, lane = threadIdx.x / nrhs;
  const bool active = lane < tp;
  const int64_t per = (Vs + kSliceChunks - 1) / kSliceChunks;
  const int64_t lo = chunk * per, hi = min(Vs, lo + per);
  cx<double> acc[kMaxPairs];
  for (int p = 0; p < A.npairs; p++) acc[p] = {0, 0};
  if (active)
    for (int64_t vs = lo + lane; vs < hi; vs += tp) {
      const int64_t e0 = ((int64_t)t * Vs + vs) * nrhs + r;
      for (int dd = 0; dd < 12; dd++) {
        const int64_t e = (int64_t)dd * N + e0;
        for (int p = 0; p < A.npairs; p++) {
          double2 av = A.a[A.ri[p]][e], bv = A.b[A.si[p]][e];
          fmac_(acc[p], cx<double>{bv.x, bv.y}, cx<double>{av.x, av.y});
        }
      }
    }
  for (int p = 0; p < A.npairs; p++) {
    sh[threadIdx.x] = active ? make_double2(acc[p].re, acc[p].im) : make_double2(0, 0);
    rhs_reduce(sh, nrhs, tp);
    if ((int)threadIdx.x < nrhs)
      partial[(((int64_t)p * nrhs + threadIdx.x) * T + t) * kSliceChunks + chunk] = sh[256 + threadIdx.x];
    __syncthreads();
  }
}

__global__ void k_slice_final(const double2* partial, int n, double2* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0, b = 0;
  for (int c = 0; c < kSliceChunks; c++) {
    double2 v = partial[(int64_t)i * kSliceChunks + c];
    a += v.x;
    b += v.y;
  }
  out[i] = make_double2(a, b);
}

void slice_pairs(Context* c, const SliceArgs& A, int64_t Vs, int T, int nrhs, double2* partial,
                 double2* out) {
  MGM_CHECK(A.npairs <= kMaxPairs && nrhs <= 256, MGM_ERR_INVALID_ARG, "slice_pairs: too many pairs");
  hipLaunchKernelGGL(k_slice_pairs, dim3(kSliceChunks, T), dim3(256), 0, c->stream, A, Vs, T, nrhs, partial);
  int n = A.npairs * nrhs * T;
  hipLaunchKernelGGL(k_slice_final, dim3(nblocks_for(n, 128)), dim3(128), 0, c->stream, partial, n, out);
  MGM_LAUNCH_CHECK();
}

// Loop reductions: out[q][g][rhs][t] = sum_{x in t} eta(x)^H Gamma_g (psi_q)(x),
// Gamma in {1, g5, gx, gy, gz, gt} of the chiral basis.
__constant__ double2 c_gamma[6][4][4];

__global__ void k_loop_gamma(LoopArgs A, int64_t Vs, int T, int nrhs, double2* partial) {
  __shared__ double2 sh[512];
  const int t = blockIdx.y;
  const int chunk = blockIdx.x;
  const int64_t N = Vs * T * nrhs;
  const int tp = 256 / nrhs;
  const int r = threadIdx.x % nrhs, lane = threadIdx.x / nrhs;
  const bool active = lane < tp;
  const int64_t per = (Vs + kSliceChunks - 1) / kSliceChunks;
  const int64_t lo = chunk * per, hi = min(Vs, lo + per);
  for (int q = 0; q < A.nvec; q++) {
    cx<double> acc[6];
    for (int g = 0; g < 6; g++) acc[g] = {0, 0};
    if (active)
      for (int64_t vs = lo + lane; vs < hi; vs += tp) {
        const int64_t e0 = ((int64_t)t * Vs + vs) * nrhs + r;
        cx<double> eta[12], psi[12];
        for (int dd = 0; dd < 12; dd++) {
          double2 ev = A.eta[(int64_t)dd * N + e0], pv = A.psi[q][(int64_t)dd * N + e0];
          eta[dd] = {ev.x, ev.y};
          psi[dd] = {pv.x, pv.y};
        }
        for (int g = 0; g < 6; g++)
          for (int s = 0; s < 4; s++)
            for (int s2 = 0; s2 < 4; s2++) {
              double2 gm = c_gamma[g][s][s2];
              if (gm.x == 0.0 && gm.y == 0.0) continue;
              for (int col = 0; col < 3; col++) {
                cx<double> gp = cx<double>{gm.x, gm.y} * psi[s2 * 3 + col];
                fmac_(acc[g], eta[s * 3 + col], gp);
              }
            }
      }
    for (int g = 0; g < 6; g++) {
      sh[threadIdx.x] = active ? make_double2(acc[g].re, acc[g].im) : make_double2(0, 0);
      rhs_reduce(sh, nrhs, tp);
      if ((int)threadIdx.x < nrhs)
        partial[((((int64_t)q * 6 + g) * nrhs + threadIdx.x) * T + t) * kSliceChunks + chunk] =
            sh[256 + threadIdx.x];
      __syncthreads();
    }
  }
}

static void host_gammas(double out[6][4][4][2]) {
  memset(out, 0, sizeof(double) * 6 * 16 * 2);
  // A_mu blocks: -i s1, -i s2, -i s3, 1
  const double A[4][2][2][2] = {
      {{{0, 0}, {0, -1}}, {{0, -1}, {0, 0}}},
      {{{0, 0}, {-1, 0}}, {{1, 0}, {0, 0}}},
      {{{0, -1}, {0, 0}}, {{0, 0}, {0, 1}}},
      {{{1, 0}, {0, 0}}, {{0, 0}, {1, 0}}},
  };
  for (int s = 0; s < 4; s++) out[0][s][s][0] = 1.0;
  for (int s = 0; s < 4; s++) out[1][s][s][0] = s < 2 ? 1.0 : -1.0;
  for (int mu = 0; mu < 4; mu++) {
    double(*g)[4][2] = out[2 + mu];
    for (int i = 0; i < 2; i++)
      for (int j = 0; j < 2; j++) {
        g[i][2 + j][0] = A[mu][i][j][0];  // upper right: A
        g[i][2 + j][1] = A[mu][i][j][1];
        g[2 + i][j][0] = A[mu][j][i][0];  // lower left: A^H
        g[2 + i][j][1] = -A[mu][j][i][1];
      }
  }
}

void loop_gamma(Context* c, const LoopArgs& A, int64_t Vs, int T, int nrhs, double2* partial, double2* out) {
  once_per_device([] {
    double g[6][4][4][2];
    host_gammas(g);
    MGM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gamma), g, sizeof(g)));
  });
  MGM_CHECK(A.nvec <= kMaxLoopVecs && nrhs <= 256, MGM_ERR_INVALID_ARG, "loop_gamma: bad arguments");
  hipLaunchKernelGGL(k_loop_gamma, dim3(kSliceChunks, T), dim3(256), 0, c->stream, A, Vs, T, nrhs, partial);
  int n = A.nvec * 6 * nrhs * T;
  hipLaunchKernelGGL(k_slice_final, dim3(nblocks_for(n, 128)), dim3(128), 0, c->stream, partial, n, out);
  MGM_LAUNCH_CHECK();
}

}  // namespace mgm
