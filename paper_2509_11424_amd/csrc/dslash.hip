// Wilson-clover operator on gfx950: clover construction and the fine dslash.
//
// Operator (the paper needs only a Gamma5-hermitian discretised Dirac
// operator with 4 spin x 3 colour dof per site, Sec. 1 and Sec. 2.1):
//   (D psi)(x) = (4 + m0) psi(x)
//     - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^H psi(x-mu)]
//     + csw (i/4) sum_{mu != nu} sigma_mu_nu F_mu_nu(x) psi(x)
// Chiral basis: g_mu = [[0, A_mu], [A_mu^H, 0]] with A_x = -i s1, A_y = -i s2,
// A_z = -i s3, A_t = 1, so (1 -/+ g_mu) psi is fixed by the half spinor
// h = u -/+ A_mu l (u, l: upper / lower spin pairs):
//   (1 - g) psi = (h, -A^H h),   (1 + g) psi = (h, A^H h).
// The dslash is HBM-bound: one thread per (site, rhs), every field stored
// component-major so each wave's loads are contiguous; the rhs index is the
// fastest so lanes of one site share (broadcast) its links and clover.
#include "fine.h"
#include "fine_dev.h"
#include "devonce.h"

namespace mgm {

// ------------------------------------------------------------ sigma table

// sigma_mu_nu = (i/2)[g_mu, g_nu] restricted to chirality chi (2 x 2), for
// the six planes mu < nu.  Upper block (i/2)(A_mu A_nu^H - A_nu A_mu^H),
// lower block (i/2)(A_mu^H A_nu - A_nu^H A_mu).
__constant__ double2 c_sigma[6][2][2][2];

static void host_sigma(double out[6][2][2][2][2]) {
  typedef double C[2];
  auto mul = [](const C* a, const C* b, C* o) {  // 2x2 complex a*b, row major
    for (int i = 0; i < 2; i++)
      for (int j = 0; j < 2; j++) {
        double re = 0, im = 0;
        for (int k = 0; k < 2; k++) {
          re += a[2 * i + k][0] * b[2 * k + j][0] - a[2 * i + k][1] * b[2 * k + j][1];
          im += a[2 * i + k][0] * b[2 * k + j][1] + a[2 * i + k][1] * b[2 * k + j][0];
        }
        o[2 * i + j][0] = re;
        o[2 * i + j][1] = im;
      }
  };
  auto dag = [](const C* a, C* o) {
    for (int i = 0; i < 2; i++)
      for (int j = 0; j < 2; j++) {
        o[2 * i + j][0] = a[2 * j + i][0];
        o[2 * i + j][1] = -a[2 * j + i][1];
      }
  };
  C A[4][4] = {
      {{0, 0}, {0, -1}, {0, -1}, {0, 0}},  // -i s1
      {{0, 0}, {-1, 0}, {1, 0}, {0, 0}},   // -i s2
      {{0, -1}, {0, 0}, {0, 0}, {0, 1}},   // -i s3
      {{1, 0}, {0, 0}, {0, 0}, {1, 0}},    // 1
  };
  int p = 0;
  for (int mu = 0; mu < 4; mu++)
    for (int nu = mu + 1; nu < 4; nu++, p++) {
      C Am_d[4], An_d[4], t1[4], t2[4];
      dag(A[mu], Am_d);
      dag(A[nu], An_d);
      for (int chi = 0; chi < 2; chi++) {
        if (chi == 0) {
          mul(A[mu], An_d, t1);
          mul(A[nu], Am_d, t2);
        } else {
          mul(Am_d, A[nu], t1);
          mul(An_d, A[mu], t2);
        }
        for (int i = 0; i < 2; i++)
          for (int j = 0; j < 2; j++) {
            double dre = t1[2 * i + j][0] - t2[2 * i + j][0];
            double dim = t1[2 * i + j][1] - t2[2 * i + j][1];
            // (i/2) * d
            out[p][chi][i][j][0] = -0.5 * dim;
            out[p][chi][i][j][1] = 0.5 * dre;
          }
      }
    }
}

// ------------------------------------------------------------- 3x3 helpers

struct M3 {
  cx<double> a[3][3];
};

__device__ __forceinline__ M3 ldU(const double2* U, int64_t V, int mu, int64_t s) {
  M3 m;
#pragma unroll
  for (int k = 0; k < 9; k++) {
    double2 v = U[(int64_t)(mu * 9 + k) * V + s];
    m.a[k / 3][k % 3] = {v.x, v.y};
  }
  return m;
}
__device__ __forceinline__ M3 mm(const M3& a, const M3& b) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) {
      cx<double> s = {0, 0};
#pragma unroll
      for (int k = 0; k < 3; k++) fma_(s, a.a[i][k], b.a[k][j]);
      c.a[i][j] = s;
    }
  return c;
}
__device__ __forceinline__ M3 dg(const M3& a) {
  M3 c;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) c.a[i][j] = conj(a.a[j][i]);
  return c;
}

__device__ __forceinline__ int64_t site_at(const Geom& g, int x, int y, int z, int t) {
  x = (x + g.X) % g.X;
  y = (y + g.Y) % g.Y;
  z = (z + g.Z) % g.Z;
  t = (t + g.T) % g.T;
  return x + (int64_t)g.X * (y + (int64_t)g.Y * (z + (int64_t)g.Z * t));
}

// --------------------------------------------------------------- clover

// One thread per site: F_mu_nu from the four plaquette leaves (all oriented
// mu then nu), F = (Q - Q^H)/8; block chi = (4+m0) 1 + csw (i/2) sum_{mu<nu}
// sigma^chi_mu_nu (x) F_mu_nu (the sum over mu != nu counts each plane twice).
__global__ void k_clover(double* __restrict__ C, const double2* __restrict__ U, Geom g, double m0,
                         double csw) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  int c[4];
  {
    int64_t q = s;
    c[0] = q % g.X; q /= g.X;
    c[1] = q % g.Y; q /= g.Y;
    c[2] = q % g.Z; q /= g.Z;
    c[3] = (int)q;
  }
  cx<double> blk[2][6][6];
  for (int chi = 0; chi < 2; chi++)
    for (int i = 0; i < 6; i++)
      for (int j = 0; j < 6; j++) blk[chi][i][j] = {i == j ? 4.0 + m0 : 0.0, 0.0};
  int p = 0;
  for (int mu = 0; mu < 4; mu++)
    for (int nu = mu + 1; nu < 4; nu++, p++) {
      auto at = [&](int dm, int dn) {
        int cc[4] = {c[0], c[1], c[2], c[3]};
        cc[mu] += dm;
        cc[nu] += dn;
        return site_at(g, cc[0], cc[1], cc[2], cc[3]);
      };
      int64_t x0 = s;
      M3 Um = ldU(U, g.V, mu, x0), Un = ldU(U, g.V, nu, x0);
      // leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
      M3 l1 = mm(mm(Um, ldU(U, g.V, nu, at(1, 0))), mm(dg(ldU(U, g.V, mu, at(0, 1))), dg(Un)));
      // leaf 2: x -> x+nu -> x+nu-mu -> x-mu -> x
      M3 l2 = mm(mm(Un, dg(ldU(U, g.V, mu, at(-1, 1)))),
                 mm(dg(ldU(U, g.V, nu, at(-1, 0))), ldU(U, g.V, mu, at(-1, 0))));
      // leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
      M3 l3 = mm(mm(dg(ldU(U, g.V, mu, at(-1, 0))), dg(ldU(U, g.V, nu, at(-1, -1)))),
                 mm(ldU(U, g.V, mu, at(-1, -1)), ldU(U, g.V, nu, at(0, -1))));
      // leaf 4: x -> x-nu -> x-nu+mu -> x+mu -> x
      M3 l4 = mm(mm(dg(ldU(U, g.V, nu, at(0, -1))), ldU(U, g.V, mu, at(0, -1))),
                 mm(ldU(U, g.V, nu, at(1, -1)), dg(Um)));
      M3 F;
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          cx<double> q = l1.a[i][j] + l2.a[i][j] + l3.a[i][j] + l4.a[i][j];
          cx<double> qd = conj(l1.a[j][i] + l2.a[j][i] + l3.a[j][i] + l4.a[j][i]);
          F.a[i][j] = 0.125 * (q - qd);
        }
      for (int chi = 0; chi < 2; chi++)
        for (int sa = 0; sa < 2; sa++)
          for (int sb = 0; sb < 2; sb++) {
            double2 sg = c_sigma[p][chi][sa][sb];
            // csw * (i/2) * sigma
            cx<double> f = {-0.5 * csw * sg.y, 0.5 * csw * sg.x};
            for (int a = 0; a < 3; a++)
              for (int b = 0; b < 3; b++) fma_(blk[chi][sa * 3 + a][sb * 3 + b], f, F.a[a][b]);
          }
    }
  for (int chi = 0; chi < 2; chi++) {
    double* o = C + (int64_t)(36 * chi) * g.V + s;
    for (int i = 0; i < 6; i++) o[(int64_t)i * g.V] = blk[chi][i][i].re;
    int q = 0;
    for (int i = 1; i < 6; i++)
      for (int j = 0; j < i; j++, q++) {
        o[(int64_t)(6 + 2 * q) * g.V] = blk[chi][i][j].re;
        o[(int64_t)(7 + 2 * q) * g.V] = blk[chi][i][j].im;
      }
  }
}

// ---------------------------------------------------------- conversions

__global__ void k_cvt_c64_c32(float2* o, const double2* in, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = make_float2((float)in[i].x, (float)in[i].y);
}
__global__ void k_cvt_c64_c16(__half2* o, const double2* in, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = __floats2half2_rn((float)in[i].x, (float)in[i].y);
}
__global__ void k_cvt_r64_r32(float* o, const double* in, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = (float)in[i];
}
__global__ void k_cvt_r64_r16(__half* o, const double* in, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = __float2half_rn((float)in[i]);
}

// ---------------------------------------------------------------- dslash

// Per-rhs block sums of the fused reductions, written to dpart[2][nrhs][block]
// (q^H in, then |q|^2).  When nq = nrhs / RB divides 64 (and nrhs <= 64),
// lane % nq fixes a thread's rhs columns: a fixed xor-shuffle tree sums each
// wave and the four wave rows are added in order.  Otherwise every thread's
// entries go through LDS and thread t < nrhs sums those of rhs t in thread
// order.  Both orders are fixed, so results are deterministic.
template <int RB>
__device__ __forceinline__ void dot_block_store(cx<double> (&dqr)[RB], double (&dqq)[RB], bool active, int r0,
                                                int nrhs, int64_t nblocks, double2* __restrict__ dpart) {
  const int nq = nrhs / RB;
  if (!active) {
#pragma unroll
    for (int j = 0; j < RB; j++) {
      dqr[j] = {0, 0};
      dqq[j] = 0;
    }
  }
  if (nrhs <= 64 && 64 % nq == 0) {
    __shared__ double2 sw_qr[4][64];
    __shared__ double sw_qq[4][64];
    for (int off = 32; off >= nq; off >>= 1) {
#pragma unroll
      for (int j = 0; j < RB; j++) {
        dqr[j].re += __shfl_xor(dqr[j].re, off, 64);
        dqr[j].im += __shfl_xor(dqr[j].im, off, 64);
        dqq[j] += __shfl_xor(dqq[j], off, 64);
      }
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane < nq) {
#pragma unroll
      for (int j = 0; j < RB; j++) {
        sw_qr[w][lane * RB + j] = make_double2(dqr[j].re, dqr[j].im);
        sw_qq[w][lane * RB + j] = dqq[j];
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < nrhs) {
      const int t = threadIdx.x;
      double a = 0, b = 0, n2 = 0;
      for (int ww = 0; ww < (int)(blockDim.x >> 6); ww++) {
        a += sw_qr[ww][t].x;
        b += sw_qr[ww][t].y;
        n2 += sw_qq[ww][t];
      }
      dpart[(int64_t)t * nblocks + blockIdx.x] = make_double2(a, b);
      dpart[(int64_t)(nrhs + t) * nblocks + blockIdx.x] = make_double2(n2, 0.0);
    }
    return;
  }
  __shared__ double2 sh_qr[256 * RB];
  __shared__ double sh_qq[256 * RB];
  __shared__ int sh_r[256 * RB];
#pragma unroll
  for (int j = 0; j < RB; j++) {
    sh_qr[threadIdx.x * RB + j] = make_double2(dqr[j].re, dqr[j].im);
    sh_qq[threadIdx.x * RB + j] = dqq[j];
    sh_r[threadIdx.x * RB + j] = active ? r0 + j : -1;
  }
  __syncthreads();
  if ((int)threadIdx.x < nrhs) {
    double a = 0, b = 0, n2 = 0;
    for (int u = 0; u < (int)blockDim.x * RB; u++)
      if (sh_r[u] == (int)threadIdx.x) {
        a += sh_qr[u].x;
        b += sh_qr[u].y;
        n2 += sh_qq[u];
      }
    dpart[(int64_t)threadIdx.x * nblocks + blockIdx.x] = make_double2(a, b);
    dpart[(int64_t)(nrhs + threadIdx.x) * nblocks + blockIdx.x] = make_double2(n2, 0.0);
  }
}

constexpr int kSlab = 4;  // time slices (one wave each) per 256-thread block

// DOT: also reduce q^H in and |q|^2 per rhs for the minimal-residual smoother
// (q = D in), written per block to dpart[2][nrhs][block] (q^H in, then |q|^2).
template <class P, bool DOT>
__global__ __launch_bounds__(256) void k_dslash(typename P::S* __restrict__ out,
                                                const typename P::S* __restrict__ in,
                                                const typename P::S* __restrict__ U,
                                                const typename P::RS* __restrict__ C, Geom g,
                                                int nrhs, int64_t nblocks, int slab,
                                                double2* __restrict__ dpart) {
  using R = typename P::R;
  const int64_t blk = xcd_block(blockIdx.x, nblocks);
  const int64_t V = g.V;
  const int64_t N = V * nrhs;
  int64_t tid;
  if (slab) {
    // Block = kSlab waves on kSlab consecutive time slices of one 64-element
    // chunk of a slice: the t-neighbours of the inner waves are loaded by
    // sibling waves of the same block at about the same time.
    const int64_t per_slice = (V / g.T) * nrhs;
    const int64_t chunks = per_slice / 64;
    const int64_t chunk = blk % chunks, tg = blk / chunks;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    tid = (tg * kSlab + w) * per_slice + chunk * 64 + lane;
  } else {
    tid = blk * blockDim.x + threadIdx.x;
  }
  // the reducing variant keeps every thread until the block reduction;
  // threads past the end compute site 0 and contribute nothing
  const bool active = tid < N;
  if (!DOT && !active) return;
  if (!active) tid = 0;
  const int64_t s = tid / nrhs;
  const int r = (int)(tid - s * nrhs);
  int c[4];
  {
    int64_t q = s;
    c[0] = (int)(q % g.X); q /= g.X;
    c[1] = (int)(q % g.Y); q /= g.Y;
    c[2] = (int)(q % g.Z); q /= g.Z;
    c[3] = (int)q;
  }
  const int64_t sy = g.X, sz = (int64_t)g.X * g.Y, st = sz * g.Z;

  cx<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; k++) acc[k] = {0, 0};
  // The eight hops run as a loop that is not unrolled, so only one
  // neighbour's spinor and link are live at a time (registers stay low and
  // occupancy high enough to cover HBM latency).
#pragma unroll 1
  for (int hop = 0; hop < 8; hop++) {
    const int mu = hop >> 1;
    const bool fwd = (hop & 1) == 0;
    const int cm = mu == 0 ? c[0] : mu == 1 ? c[1] : mu == 2 ? c[2] : c[3];
    const int ex = mu == 0 ? g.X : mu == 1 ? g.Y : mu == 2 ? g.Z : g.T;
    const int64_t sd = mu == 0 ? 1 : mu == 1 ? sy : mu == 2 ? sz : st;
    const bool wrap = fwd ? (cm == ex - 1) : (cm == 0);
    const int64_t span = (int64_t)(ex - 1) * sd;
    const int64_t sn = fwd ? (wrap ? s - span : s + sd) : (wrap ? s + span : s - sd);
    // -1/2 (1 -/+ g_mu), times -1 on hops across the time boundary
    const R f = (mu == 3 && wrap && g.antiperiodic) ? (R)0.5 : (R)-0.5;
    const R sg = fwd ? (R)-1 : (R)1;  // half spinor h = u + sg * A_mu l
    const int64_t e = sn * nrhs + r;
    cx<R> h[2][3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      cx<R> u0 = P::ld(in, (int64_t)(0 * 3 + a) * N + e), u1 = P::ld(in, (int64_t)(1 * 3 + a) * N + e);
      cx<R> l0 = P::ld(in, (int64_t)(2 * 3 + a) * N + e), l1 = P::ld(in, (int64_t)(3 * 3 + a) * N + e);
      cx<R> a0, a1;
      A_times(mu, l0, l1, a0, a1);
      h[0][a] = u0 + sg * a0;
      h[1][a] = u1 + sg * a1;
    }
    // forward: U_mu(x) h ; backward: U_mu(x - mu)^H h
    const typename P::S* Ub = U + (int64_t)(mu * 9) * V + (fwd ? s : sn);
    cx<R> Um[3][3];
#pragma unroll
    for (int k = 0; k < 9; k++) Um[k / 3][k % 3] = P::ld(Ub, (int64_t)k * V);
#pragma unroll
    for (int a = 0; a < 3; a++) {
      cx<R> g0 = {0, 0}, g1 = {0, 0};
      if (fwd) {
#pragma unroll
        for (int b = 0; b < 3; b++) {
          fma_(g0, Um[a][b], h[0][b]);
          fma_(g1, Um[a][b], h[1][b]);
        }
      } else {
#pragma unroll
        for (int b = 0; b < 3; b++) {  // (U^H)_{ab} = conj(U_{ba})
          fmac_(g0, Um[b][a], h[0][b]);
          fmac_(g1, Um[b][a], h[1][b]);
        }
      }
      cx<R> d0, d1;
      Ad_times(mu, g0, g1, d0, d1);  // lower spins: -A^H g (forward), +A^H g (backward)
      const R fs = f * sg;
      axpy_(acc[0 * 3 + a], f, g0);
      axpy_(acc[1 * 3 + a], f, g1);
      axpy_(acc[2 * 3 + a], fs, d0);
      axpy_(acc[3 * 3 + a], fs, d1);
    }
  }
  // site-local term: clover blocks with the mass folded into the diagonal
  cx<double> dqr = {0, 0};
  double dqq = 0;
#pragma unroll 1
  for (int chi = 0; chi < 2; chi++) {
    cx<R> p[6], q[6];
#pragma unroll
    for (int k = 0; k < 6; k++) p[k] = P::ld(in, (int64_t)(6 * chi + k) * N + tid);
    clover_block<P>(C, V, s, chi, p, q);
#pragma unroll
    for (int k = 0; k < 6; k++) {
      cx<R> o;
      if (chi == 0) o = acc[k] = acc[k] + q[k];
      else o = acc[6 + k] = acc[6 + k] + q[k];
      if (DOT) {
        // the rounded stored value enters the dots
        typename P::S st_;
        P::st(&st_, 0, o);
        const cx<R> os = P::ld(&st_, 0);
        fmac_(dqr, cx<double>{(double)os.re, (double)os.im}, cx<double>{(double)p[k].re, (double)p[k].im});
        dqq += (double)os.re * os.re + (double)os.im * os.im;
      }
    }
  }
  if (active) {
#pragma unroll
    for (int k = 0; k < 12; k++) P::st(out, (int64_t)k * N + tid, acc[k]);
  }
  if (DOT) {
    cx<double> qr1[1] = {dqr};
    double qq1[1] = {dqq};
    dot_block_store<1>(qr1, qq1, active, r, nrhs, nblocks, dpart);
  }
}

// Variant for FP32/FP16 with an even rhs count: one thread computes RB = 2
// consecutive right-hand sides of one site, so the links, clover entries and
// index arithmetic are shared by the two columns and the spinor loads become
// 16-byte (FP32) or 8-byte (FP16) vector loads.  Same block order, DOT
// reduction and output as k_dslash.
template <class P, bool DOT, int RB>
__global__ __launch_bounds__(256) void k_dslash_rb(typename P::S* __restrict__ out,
                                                const typename P::S* __restrict__ in,
                                                const typename P::S* __restrict__ U,
                                                const typename P::RS* __restrict__ C, Geom g,
                                                int nrhs, int64_t nblocks, int slab,
                                                double2* __restrict__ dpart) {
  using R = typename P::R;
  const int64_t blk = xcd_block(blockIdx.x, nblocks);
  const int64_t V = g.V;
  const int64_t N = V * nrhs;       // elements per dof plane
  const int nq = nrhs / RB;         // threads per site
  const int64_t NT = V * nq;        // threads in the grid that carry work
  int64_t tid;
  if (slab) {
    // Block = kSlab waves on kSlab consecutive time slices of one 64-thread
    // chunk of a slice: the t-neighbours of the inner waves are loaded by
    // sibling waves of the same block at about the same time.
    const int64_t per_slice = (V / g.T) * nq;
    const int64_t chunks = per_slice / 64;
    const int64_t chunk = blk % chunks, tg = blk / chunks;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    tid = (tg * kSlab + w) * per_slice + chunk * 64 + lane;
  } else {
    tid = blk * blockDim.x + threadIdx.x;
  }
  // the reducing variant keeps every thread until the block reduction;
  // threads past the end compute site 0 and contribute nothing
  const bool active = tid < NT;
  if (!DOT && !active) return;
  if (!active) tid = 0;
  const int64_t s = tid / nq;
  const int r0 = (int)(tid - s * nq) * RB;
  const int64_t es = s * nrhs + r0;  // this thread's first element in a plane
  int c[4];
  {
    int64_t q = s;
    c[0] = (int)(q % g.X); q /= g.X;
    c[1] = (int)(q % g.Y); q /= g.Y;
    c[2] = (int)(q % g.Z); q /= g.Z;
    c[3] = (int)q;
  }
  const int64_t sy = g.X, sz = (int64_t)g.X * g.Y, st = sz * g.Z;

  cx<R> acc[12][RB];
#pragma unroll
  for (int k = 0; k < 12; k++)
#pragma unroll
    for (int j = 0; j < RB; j++) acc[k][j] = {0, 0};
  // The eight hops run as a loop that is not unrolled, so only one
  // neighbour's spinor and link are live at a time (registers stay low and
  // occupancy high enough to cover HBM latency).
#pragma unroll 1
  for (int hop = 0; hop < 8; hop++) {
    const int mu = hop >> 1;
    const bool fwd = (hop & 1) == 0;
    const int cm = mu == 0 ? c[0] : mu == 1 ? c[1] : mu == 2 ? c[2] : c[3];
    const int ex = mu == 0 ? g.X : mu == 1 ? g.Y : mu == 2 ? g.Z : g.T;
    const int64_t sd = mu == 0 ? 1 : mu == 1 ? sy : mu == 2 ? sz : st;
    const bool wrap = fwd ? (cm == ex - 1) : (cm == 0);
    const int64_t span = (int64_t)(ex - 1) * sd;
    const int64_t sn = fwd ? (wrap ? s - span : s + sd) : (wrap ? s + span : s - sd);
    // -1/2 (1 -/+ g_mu), times -1 on hops across the time boundary
    const R f = (mu == 3 && wrap && g.antiperiodic) ? (R)0.5 : (R)-0.5;
    const R sg = fwd ? (R)-1 : (R)1;  // half spinor h = u + sg * A_mu l
    const int64_t e = sn * nrhs + r0;
    cx<R> h[2][3][RB];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      cx<R> u0[RB], u1[RB], l0[RB], l1[RB];
      P::template ldv<RB>(in, (int64_t)(0 * 3 + a) * N + e, u0);
      P::template ldv<RB>(in, (int64_t)(1 * 3 + a) * N + e, u1);
      P::template ldv<RB>(in, (int64_t)(2 * 3 + a) * N + e, l0);
      P::template ldv<RB>(in, (int64_t)(3 * 3 + a) * N + e, l1);
#pragma unroll
      for (int j = 0; j < RB; j++) {
        cx<R> a0, a1;
        A_times(mu, l0[j], l1[j], a0, a1);
        h[0][a][j] = u0[j] + sg * a0;
        h[1][a][j] = u1[j] + sg * a1;
      }
    }
    // forward: U_mu(x) h ; backward: U_mu(x - mu)^H h
    const typename P::S* Ub = U + (int64_t)(mu * 9) * V + (fwd ? s : sn);
    cx<R> Um[3][3];
#pragma unroll
    for (int k = 0; k < 9; k++) Um[k / 3][k % 3] = P::ld(Ub, (int64_t)k * V);
#pragma unroll
    for (int j = 0; j < RB; j++)
#pragma unroll
      for (int a = 0; a < 3; a++) {
        cx<R> g0 = {0, 0}, g1 = {0, 0};
        if (fwd) {
#pragma unroll
          for (int b = 0; b < 3; b++) {
            fma_(g0, Um[a][b], h[0][b][j]);
            fma_(g1, Um[a][b], h[1][b][j]);
          }
        } else {
#pragma unroll
          for (int b = 0; b < 3; b++) {  // (U^H)_{ab} = conj(U_{ba})
            fmac_(g0, Um[b][a], h[0][b][j]);
            fmac_(g1, Um[b][a], h[1][b][j]);
          }
        }
        cx<R> d0, d1;
        Ad_times(mu, g0, g1, d0, d1);  // lower spins: -A^H g (forward), +A^H g (backward)
        const R fs = f * sg;
        axpy_(acc[0 * 3 + a][j], f, g0);
        axpy_(acc[1 * 3 + a][j], f, g1);
        axpy_(acc[2 * 3 + a][j], fs, d0);
        axpy_(acc[3 * 3 + a][j], fs, d1);
      }
  }
  // site-local term: clover blocks with the mass folded into the diagonal
  cx<double> dqr[RB];
  double dqq[RB];
#pragma unroll
  for (int j = 0; j < RB; j++) {
    dqr[j] = {0, 0};
    dqq[j] = 0;
  }
#pragma unroll 1
  for (int chi = 0; chi < 2; chi++) {
    cx<R> pv[6][RB];
#pragma unroll
    for (int k = 0; k < 6; k++) P::template ldv<RB>(in, (int64_t)(6 * chi + k) * N + es, pv[k]);
#pragma unroll
    for (int j = 0; j < RB; j++) {
      cx<R> x6[6], q6[6];
#pragma unroll
      for (int k = 0; k < 6; k++) x6[k] = pv[k][j];
      clover_block<P>(C, V, s, chi, x6, q6);
#pragma unroll
      for (int k = 0; k < 6; k++) {
        cx<R> o;
        if (chi == 0) o = acc[k][j] = acc[k][j] + q6[k];
        else o = acc[6 + k][j] = acc[6 + k][j] + q6[k];
        if (DOT) {
          // the rounded stored value enters the dots
          typename P::S st_;
          P::st(&st_, 0, o);
          const cx<R> os = P::ld(&st_, 0);
          fmac_(dqr[j], cx<double>{(double)os.re, (double)os.im}, cx<double>{(double)x6[k].re, (double)x6[k].im});
          dqq[j] += (double)os.re * os.re + (double)os.im * os.im;
        }
      }
    }
  }
  if (active) {
#pragma unroll
    for (int k = 0; k < 12; k++) P::template stv<RB>(out, (int64_t)k * N + es, acc[k]);
  }
  if (DOT) dot_block_store<RB>(dqr, dqq, active, r0, nrhs, nblocks, dpart);
}

// ------------------------------------------------- plane-marching dslash
//
// One block owns a tile of TY full x-rows of one time slice, for a group of
// nbr consecutive right-hand sides, and marches through zs consecutive
// z-planes.  Each plane of the input is read
// from HBM once by its owner: it is staged in LDS, with one halo row on each
// side in y, for the x- and y-hops; kept in registers as the centre of the
// next step; and its backward z-hop contribution to the next plane is formed
// while it is in registers.  The t-hops read the same tile of the adjacent
// time slices, which belong to the neighbouring blocks in block order (the
// time slice is the fastest block index), so they are loaded by blocks
// resident on the same XCD; they too are formed one step early, in the step
// in which the owners of those slices load the plane as their next one, so
// the rows are still in L2 (a step later, the streams of the 32 blocks on an
// XCD have moved more than its 4 MB of L2 through it).  Every hop and the
// clover term use the same arithmetic as k_dslash; the terms are summed in
// another order (the backward z and the t hops first, as they are formed one
// step early, and the forward z hop last, after the loads of the next plane
// are in flight), so the two kernels agree to rounding.

// gg = U h (forward) or U^H h (backward) for the half spinor h = u -/+ A_mu l
// of ps
template <class P>
__device__ __forceinline__ void hop_half(int mu, bool fwd, const cx<typename P::R> (&ps)[12],
                                         const cx<typename P::R> (&Um)[3][3], cx<typename P::R> (&gg)[2][3]) {
  using R = typename P::R;
  const R sg = fwd ? (R)-1 : (R)1;
  cx<R> h[2][3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    cx<R> a0, a1;
    A_times(mu, ps[6 + a], ps[9 + a], a0, a1);
    h[0][a] = ps[a] + sg * a0;
    h[1][a] = ps[3 + a] + sg * a1;
  }
#pragma unroll
  for (int a = 0; a < 3; a++) {
    cx<R> g0 = {0, 0}, g1 = {0, 0};
    if (fwd) {
#pragma unroll
      for (int b = 0; b < 3; b++) {
        fma_(g0, Um[a][b], h[0][b]);
        fma_(g1, Um[a][b], h[1][b]);
      }
    } else {
#pragma unroll
      for (int b = 0; b < 3; b++) {
        fmac_(g0, Um[b][a], h[0][b]);
        fmac_(g1, Um[b][a], h[1][b]);
      }
    }
    gg[0][a] = g0;
    gg[1][a] = g1;
  }
}

// acc += f (1 -/+ g_mu) expansion of gg (f = -1/2, or +1/2 across the
// antiperiodic time boundary)
template <class P>
__device__ __forceinline__ void hop_add(int mu, bool fwd, typename P::R f, const cx<typename P::R> (&gg)[2][3],
                                        cx<typename P::R> (&acc)[12]) {
  using R = typename P::R;
  const R fs = fwd ? -f : f;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    cx<R> d0, d1;
    Ad_times(mu, gg[0][a], gg[1][a], d0, d1);
    axpy_(acc[0 * 3 + a], f, gg[0][a]);
    axpy_(acc[1 * 3 + a], f, gg[1][a]);
    axpy_(acc[2 * 3 + a], fs, d0);
    axpy_(acc[3 * 3 + a], fs, d1);
  }
}

// Buffer loads for the marching kernel: one SGPR descriptor per array and a
// 32-bit byte offset per lane (plus a uniform offset per dof plane), so the
// twelve planes of a spinor share one address register.  Every array it
// reads is below 4 GiB (checked on the host); an offset past the end would
// read zero, never fault.
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <class P>
struct BufIO;
template <>
struct BufIO<F32> {
  using S = float2;
  static constexpr uint32_t SB = 8, RB = 4;  // bytes of a complex / real element
  template <int AUX = 0>
  __device__ __forceinline__ static S raw(Rsrc r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, AUX));
  }
  __device__ __forceinline__ static cx<float> cvt(S v) { return {v.x, v.y}; }
  __device__ __forceinline__ static float re(Rsrc r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
  }
  template <int AUX = 0>
  __device__ __forceinline__ static void st(Rsrc r, uint32_t vo, uint32_t so, cx<float> v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), make_float2(v.re, v.im)), r, (int)vo, (int)so, AUX);
  }
};
template <>
struct BufIO<F16> {
  using S = __half2;
  static constexpr uint32_t SB = 4, RB = 2;
  template <int AUX = 0>
  __device__ __forceinline__ static S raw(Rsrc r, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, AUX));
  }
  __device__ __forceinline__ static cx<float> cvt(S v) {
    const float2 f = __half22float2(v);
    return {f.x, f.y};
  }
  __device__ __forceinline__ static float re(Rsrc r, uint32_t vo, uint32_t so) {
    return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0)));
  }
  template <int AUX = 0>
  __device__ __forceinline__ static void st(Rsrc r, uint32_t vo, uint32_t so, cx<float> v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, __floats2half2_rn(v.re, v.im)), r, (int)vo,
                                          (int)so, AUX);
  }
};

// link U_mu at the site whose byte offset (in a link plane) is vo
template <class P>
__device__ __forceinline__ void buf_link(Rsrc ru, uint32_t plane_b, int mu, uint32_t vo,
                                         cx<typename P::R> (&Um)[3][3]) {
#pragma unroll
  for (int k = 0; k < 9; k++)
    Um[k / 3][k % 3] = BufIO<P>::cvt(BufIO<P>::raw(ru, vo, (uint32_t)(mu * 9 + k) * plane_b));
}

// Hermitian 6x6 clover block times p (same arithmetic as clover_block)
template <class P>
__device__ __forceinline__ void buf_clover(Rsrc rc, uint32_t plane_b, uint32_t vo, int chi,
                                           const cx<typename P::R>* x, cx<typename P::R>* y) {
  using R = typename P::R;
  const uint32_t b0 = (uint32_t)(36 * chi) * plane_b;
#pragma unroll
  for (int i = 0; i < 6; i++) {
    R d = BufIO<P>::re(rc, vo, b0 + (uint32_t)i * plane_b);
    y[i] = d * x[i];
  }
  int q = 0;
#pragma unroll
  for (int i = 1; i < 6; i++)
#pragma unroll
    for (int j = 0; j < i; j++, q++) {
      cx<R> cij = {BufIO<P>::re(rc, vo, b0 + (uint32_t)(6 + 2 * q) * plane_b),
                   BufIO<P>::re(rc, vo, b0 + (uint32_t)(7 + 2 * q) * plane_b)};
      fma_(y[i], cij, x[j]);
      fmac_(y[j], cij, x[i]);
    }
}

// ------------------------------------------------ packed FP16 arithmetic
//
// The FP16 marching kernel can keep the spinors and links in their storage
// format: the half spinor h = u -/+ A_mu l is formed with FP16 adds (one
// rounding to FP16, like the stored input), and every complex product with a
// link or clover entry is a pair of v_dot2_f32_f16 (two FP16 products, exact
// in FP32, added to an FP32 accumulator): re(U h) = dot2(U, (h.re, -h.im)),
// im(U h) = dot2(U, (h.im, h.re)); re(conj(U) h) = dot2(U, h),
// im(conj(U) h) = dot2(U, (h.im, -h.re)).  No conversion of links, clover
// entries or neighbour spinors, half the multiply instructions of the FP32
// form, and half the registers for the neighbour spinor.
typedef _Float16 hv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ hv2 hv(__half2 v) { return __builtin_bit_cast(hv2, v); }
__device__ __forceinline__ float dot2(hv2 a, hv2 b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }
__device__ __forceinline__ hv2 hmul_i(hv2 z) { return hv2{(_Float16)-z.y, z.x}; }
__device__ __forceinline__ hv2 hmul_mi(hv2 z) { return hv2{z.y, (_Float16)-z.x}; }

// h = u -/+ A_mu l (fwd: minus) in FP16
__device__ __forceinline__ void half_spinor_pk(int mu, bool fwd, const hv2 (&ps)[12], hv2 (&h)[2][3]) {
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const hv2 l0 = ps[6 + a], l1 = ps[9 + a];
    hv2 o0, o1;
    switch (mu) {
      case 0: o0 = hmul_mi(l1); o1 = hmul_mi(l0); break;  // -i s1
      case 1: o0 = -l1; o1 = l0; break;                   // -i s2
      case 2: o0 = hmul_mi(l0); o1 = hmul_i(l1); break;   // -i s3
      default: o0 = l0; o1 = l1; break;                   // 1
    }
    h[0][a] = fwd ? ps[a] - o0 : ps[a] + o0;
    h[1][a] = fwd ? ps[3 + a] - o1 : ps[3 + a] + o1;
  }
}

// gg = U h (fwd) or U^H h (bwd) with FP32 sums of FP16 products
__device__ __forceinline__ void link_mul_pk(bool fwd, const hv2 (&U)[3][3], const hv2 (&h)[2][3],
                                            cx<float> (&gg)[2][3]) {
  if (fwd) {
    hv2 hn[2][3], hs[2][3];
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
      for (int b = 0; b < 3; b++) {
        hn[s][b] = hv2{h[s][b].x, (_Float16)-h[s][b].y};
        hs[s][b] = hv2{h[s][b].y, h[s][b].x};
      }
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int s = 0; s < 2; s++) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int b = 0; b < 3; b++) {
          re = dot2(U[a][b], hn[s][b], re);
          im = dot2(U[a][b], hs[s][b], im);
        }
        gg[s][a] = {re, im};
      }
  } else {
    hv2 hm[2][3];
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
      for (int b = 0; b < 3; b++) hm[s][b] = hv2{h[s][b].y, (_Float16)-h[s][b].x};
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int s = 0; s < 2; s++) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int b = 0; b < 3; b++) {
          re = dot2(U[b][a], h[s][b], re);
          im = dot2(U[b][a], hm[s][b], im);
        }
        gg[s][a] = {re, im};
      }
  }
}

// the nine links U_mu at byte offset vo, in their FP16 storage
__device__ __forceinline__ void buf_link_pk(Rsrc ru, uint32_t plane_b, int mu, uint32_t vo, hv2 (&U)[3][3]) {
#pragma unroll
  for (int k = 0; k < 9; k++)
    U[k / 3][k % 3] = __builtin_bit_cast(hv2, __builtin_amdgcn_raw_buffer_load_b32(ru, (int)vo,
                                                                                 (int)((uint32_t)(mu * 9 + k) * plane_b), 0));
}

// Hermitian 6x6 clover block (FP16 planes: 6 diagonal reals, then the 15
// entries below the diagonal as (re, im) plane pairs) times x: diagonal in
// FP32, off-diagonal products by dot2
__device__ __forceinline__ void buf_clover_pk(Rsrc rc, uint32_t plane_b, uint32_t vo, int chi, const hv2 (&x)[6],
                                              cx<float> (&y)[6]) {
  const uint32_t b0 = (uint32_t)(36 * chi) * plane_b;
  auto ld16 = [&](uint32_t so) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rc, (int)vo, (int)so, 0));
  };
  hv2 xn[6], xs[6], xm[6];
#pragma unroll
  for (int i = 0; i < 6; i++) {
    const float d = (float)ld16(b0 + (uint32_t)i * plane_b);
    y[i] = {d * (float)x[i].x, d * (float)x[i].y};
    xn[i] = hv2{x[i].x, (_Float16)-x[i].y};
    xs[i] = hv2{x[i].y, x[i].x};
    xm[i] = hv2{x[i].y, (_Float16)-x[i].x};
  }
  int q = 0;
#pragma unroll
  for (int i = 1; i < 6; i++)
#pragma unroll
    for (int j = 0; j < i; j++, q++) {
      const hv2 c = hv2{ld16(b0 + (uint32_t)(6 + 2 * q) * plane_b), ld16(b0 + (uint32_t)(7 + 2 * q) * plane_b)};
      y[i].re = dot2(c, xn[j], y[i].re);  // c x_j
      y[i].im = dot2(c, xs[j], y[i].im);
      y[j].re = dot2(c, x[i], y[j].re);   // conj(c) x_i
      y[j].im = dot2(c, xm[i], y[j].im);
    }
}

// gg of one hop from the twelve stored components of the neighbour spinor
// and the link at byte offset lvo: FP32 arithmetic on converted values, or
// (PK, FP16 storage only) the packed FP16 form above
template <class P, bool PK>
__device__ __forceinline__ void hop_raw(const typename P::S (&raw)[12], int mu, bool fwd, Rsrc ru, uint32_t upb,
                                        uint32_t lvo, cx<typename P::R> (&gg)[2][3]) {
  if constexpr (PK) {
    hv2 ps[12];
#pragma unroll
    for (int k = 0; k < 12; k++) ps[k] = hv(raw[k]);
    hv2 U[3][3], h[2][3];
    buf_link_pk(ru, upb, mu, lvo, U);
    half_spinor_pk(mu, fwd, ps, h);
    link_mul_pk(fwd, U, h, gg);
  } else {
    cx<typename P::R> ps[12], Um[3][3];
#pragma unroll
    for (int k = 0; k < 12; k++) ps[k] = BufIO<P>::cvt(raw[k]);
    buf_link<P>(ru, upb, mu, lvo, Um);
    hop_half<P>(mu, fwd, ps, Um, gg);
  }
}

// Launch: blockDim = X * TY * nbr (a multiple of 64, at most MAXT), grid =
// (nrhs / nbr) * T * (Y / TY) * (Z / zs), dynamic LDS = 2 * 12 * (TY + 2) * X *
// nbr elements of P::S (at least the DOT reduction's 16 * 64 * 24 bytes);
// nbr divides nrhs and 64; TY is even; 12 * V * nrhs spinor elements, the
// links and the clover each below 4 GiB.
//
// MR (with DOT): one step of the minimal-residual smoother with the step
// length of the previous step (Richardson with lagged MR lengths).  `in`
// holds r, `wqr`/`wqq` the dots of the previous step, omega = wqr / wqq per
// rhs (0 where wqq is 0).  q = D r is not stored: the owner of a site
// writes r - omega q to `out` and updates x += omega r in place in `xio`;
// the dots are those of (q, r) (q unrounded), which give the next step's
// length.  in, out
// and xio are distinct arrays.
template <class P, bool DOT, bool MR, int TY, int MAXT, bool PK = false>
__global__ __launch_bounds__(MAXT) void k_dslash_march(typename P::S* __restrict__ out,
                                                       const typename P::S* __restrict__ in,
                                                       const typename P::S* __restrict__ U,
                                                       const typename P::RS* __restrict__ C, Geom g, int nrhs,
                                                       int nbr, int zs, int64_t nblocks,
                                                       double2* __restrict__ dpart,
                                                       typename P::S* __restrict__ xio,
                                                       const double2* __restrict__ wqr,
                                                       const double* __restrict__ wqq) {
  using R = typename P::R;
  using S = typename P::S;
  using IO = BufIO<P>;
  static_assert(!MR || DOT, "the smoother step also produces the next dots");
  static_assert(!PK || std::is_same<P, F16>::value, "packed arithmetic needs FP16 storage");
  extern __shared__ __align__(16) unsigned char march_smem[];
  // two plane buffers [2][12][TY + 2][X * nbr]: step i reads buffer i % 2
  // and stages the next plane into the other, so one barrier per step
  S* pl = reinterpret_cast<S*>(march_smem);
  constexpr int kRows = TY + 2;
  const uint32_t V = (uint32_t)g.V, N = V * (uint32_t)nrhs;
  const uint32_t spb = N * IO::SB;   // bytes per spinor dof plane
  const uint32_t upb = V * IO::SB;   // bytes per link plane
  const uint32_t cpb = V * IO::RB;   // bytes per clover plane
  const Rsrc rin = make_rsrc(in, 12 * spb), rout = make_rsrc(out, 12 * spb);
  const Rsrc ru = make_rsrc(U, 36 * upb), rc = make_rsrc(C, 72 * cpb);
  const int rowlen = g.X * nbr;
  const int64_t blk = xcd_block(blockIdx.x, nblocks);
  const int nsub = nrhs / nbr;
  const int rb0 = (int)(blk % nsub) * nbr;  // first rhs of the group
  const int t = (int)((blk / nsub) % g.T);
  const int rest = (int)(blk / nsub / g.T);
  const int ntile = g.Y / TY;
  const int y0 = (rest % ntile) * TY;
  const int z0 = (rest / ntile) * zs;
  const int tid = threadIdx.x;
  const int rl = tid % nbr, r = rb0 + rl;
  const int col = tid % rowlen;  // x * nbr + rl
  const int xs = col / nbr;
  const int yl = tid / rowlen;
  const int y = y0 + yl;
  const uint32_t sy = g.X, sz = (uint32_t)g.X * g.Y, st = sz * g.Z;
  const int xp = xs == g.X - 1 ? 0 : xs + 1, xm = xs == 0 ? g.X - 1 : xs - 1;
  const int ym = y == 0 ? g.Y - 1 : y - 1;
  const int tp = t == g.T - 1 ? 0 : t + 1, tm = t == 0 ? g.T - 1 : t - 1;
  const R ftp = (t == g.T - 1 && g.antiperiodic) ? (R)0.5 : (R)-0.5;
  const R ftm = (t == 0 && g.antiperiodic) ? (R)0.5 : (R)-0.5;
  const int hy0 = y0 == 0 ? g.Y - 1 : y0 - 1, hy1 = y0 + TY == g.Y ? 0 : y0 + TY;
  const uint32_t rowoff = (uint32_t)y * sy + xs;  // (x, y) part of a site index
  // LDS element of dof k, LDS row lr, column c
  const int plane_elems = 12 * kRows * rowlen;
  auto lidx = [&](int k, int lr, int c) { return (k * kRows + lr) * rowlen + c; };
  // Halo rows: 12 dof x 2 rows = 24 row-planes; thread (yl, col) stages
  // row-plane q = yl + TY j (all q < 24) at its own column, i.e. dof
  // yl / 2 + (TY / 2) j of halo row yl % 2 (TY is even).
  const int hrow = yl & 1, hk0 = yl >> 1;
  const uint32_t hyoff = (uint32_t)(hrow ? hy1 : hy0) * sy;
  // smoother step: lagged step length and the x array (the descriptor
  // aliases the input when unused)
  const Rsrc rx = make_rsrc(MR ? (const void*)xio : (const void*)in, 12 * spb);
  cx<R> om = {0, 0};
  if (MR) {
    const double d = wqq[r];
    if (d > 0.0) om = {(R)(wqr[r].x / d), (R)(wqr[r].y / d)};
  }
  auto stage_halo = [&](int zz, S* buf) {
    // the per-thread dof offset goes into the lane offset, the per-j one
    // into the uniform offset
    const uint32_t vo = (((uint32_t)zz * sz + (uint32_t)t * st + hyoff + xs) * nrhs + r) * IO::SB +
                        (uint32_t)hk0 * spb;
#pragma unroll
    for (int j = 0; j < (24 + TY - 1) / TY; j++) {
      const int k = hk0 + (TY / 2) * j;
      if (24 % TY == 0 || k < 12)
        buf[lidx(k, hrow ? kRows - 1 : 0, col)] = IO::raw(rin, vo, (uint32_t)((TY / 2) * j) * spb);
    }
  };
  // t hops of plane zz from the adjacent slices into acc.  In the smoother
  // step they are formed one step early (at the end of the step before plane
  // zz), when the owners of the adjacent slices load plane zz as their next
  // plane: both reads of those rows fall into the same step, and the second
  // finds them in L2.  The other forms keep them in their own step (their
  // dot accumulators leave no registers for the early form).
  constexpr bool kTEarly = MR;
  auto t_hops = [&](int zz, cx<R>(&a)[12]) {
    const uint32_t s_own = (uint32_t)zz * sz + (uint32_t)t * st + rowoff;
#pragma unroll 1
    for (int hop = 0; hop < 2; hop++) {
      const bool fwd = hop == 0;
      const uint32_t sn = (uint32_t)zz * sz + (uint32_t)(fwd ? tp : tm) * st + rowoff;
      S ps[12];
      cx<R> gg[2][3];
#pragma unroll
      for (int k = 0; k < 12; k++) ps[k] = IO::raw(rin, (sn * nrhs + r) * IO::SB, (uint32_t)k * spb);
      hop_raw<P, PK>(ps, 3, fwd, ru, upb, (fwd ? s_own : sn) * IO::SB, gg);
      hop_add<P>(3, fwd, fwd ? ftp : ftm, gg, a);
    }
  };
  // The accumulator of a plane starts as the backward z-hop contribution of
  // the plane before it, formed while that plane is in registers, plus the
  // plane's t hops.
  cx<R> acc[12];
  {
    const int zm = z0 == 0 ? g.Z - 1 : z0 - 1;
    const uint32_t sm = (uint32_t)zm * sz + (uint32_t)t * st + rowoff;
    S pm[12];
    cx<R> gg[2][3];
#pragma unroll
    for (int k = 0; k < 12; k++) pm[k] = IO::raw(rin, (sm * nrhs + r) * IO::SB, (uint32_t)k * spb);
    hop_raw<P, PK>(pm, 2, false, ru, upb, sm * IO::SB, gg);
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = {0, 0};
    hop_add<P>(2, false, (R)-0.5, gg, acc);
    if (kTEarly) t_hops(z0, acc);
    const uint32_t s0 = (uint32_t)z0 * sz + (uint32_t)t * st + rowoff;
#pragma unroll
    for (int k = 0; k < 12; k++) {
      const S rv = IO::raw(rin, (s0 * nrhs + r) * IO::SB, (uint32_t)k * spb);
      pl[lidx(k, yl + 1, col)] = rv;
    }
    stage_halo(z0, pl);
  }
  cx<double> dqr = {0, 0};
  double dqq = 0;
#pragma unroll 1
  for (int i = 0; i < zs; i++) {
    const int z = z0 + i;
    const int zp = z == g.Z - 1 ? 0 : z + 1;
    const uint32_t s = (uint32_t)z * sz + (uint32_t)t * st + rowoff;
    S* const cur = pl + (i & 1) * plane_elems;  // plane z
    S* const nxt = pl + ((i & 1) ^ 1) * plane_elems;  // plane z + 1, staged during this step
    __syncthreads();  // plane z staged; every read of the other buffer done
    // x and y hops from LDS
#pragma unroll 1
    for (int hop = 0; hop < 4; hop++) {
      const int mu = hop >> 1;
      const bool fwd = (hop & 1) == 0;
      int lrow, lcol;
      uint32_t ls;  // site owning the link
      if (mu == 0) {
        lrow = yl + 1;
        lcol = (fwd ? xp : xm) * nbr + rl;
        ls = fwd ? s : s - xs + xm;
      } else {
        lrow = fwd ? yl + 2 : yl;
        lcol = col;
        ls = fwd ? s : s + (uint32_t)(ym - y) * sy;
      }
      S ps[12];
      cx<R> gg[2][3];
#pragma unroll
      for (int k = 0; k < 12; k++) ps[k] = cur[lidx(k, lrow, lcol)];
      hop_raw<P, PK>(ps, mu, fwd, ru, upb, ls * IO::SB, gg);
      hop_add<P>(mu, fwd, (R)-0.5, gg, acc);
    }
    if (!kTEarly) t_hops(z, acc);
    // next plane (kept raw for staging); its loads overlap the clover term
    S nx[12];
    {
      const uint32_t vn = (((uint32_t)zp * sz + (uint32_t)t * st + rowoff) * nrhs + r) * IO::SB;
#pragma unroll
      for (int k = 0; k < 12; k++) nx[k] = IO::raw(rin, vn, (uint32_t)k * spb);
    }
    // site-local term with the centre from LDS
#pragma unroll 1
    for (int chi = 0; chi < 2; chi++) {
      cx<R> q6[6];
      if constexpr (PK) {
        hv2 x6[6];
#pragma unroll
        for (int k = 0; k < 6; k++) x6[k] = hv(cur[lidx(6 * chi + k, yl + 1, col)]);
        buf_clover_pk(rc, cpb, s * IO::RB, chi, x6, q6);
      } else {
        cx<R> p6[6];
#pragma unroll
        for (int k = 0; k < 6; k++) p6[k] = IO::cvt(cur[lidx(6 * chi + k, yl + 1, col)]);
        buf_clover<P>(rc, cpb, s * IO::RB, chi, p6, q6);
      }
#pragma unroll
      for (int k = 0; k < 6; k++) {
        if (chi == 0) acc[k] = acc[k] + q6[k];
        else acc[6 + k] = acc[6 + k] + q6[k];
      }
    }
    // forward z hop from the next plane
    {
      cx<R> gg[2][3];
      hop_raw<P, PK>(nx, 2, true, ru, upb, s * IO::SB, gg);
      hop_add<P>(2, true, (R)-0.5, gg, acc);
    }
    // stage the next plane (own rows from the registers, halo rows loaded)
    if (i + 1 < zs) {
      const uint32_t vn = (((uint32_t)zp * sz + (uint32_t)t * st + rowoff) * nrhs + r) * IO::SB;
#pragma unroll
      for (int k = 0; k < 12; k++) nxt[lidx(k, yl + 1, col)] = nx[k];
      stage_halo(zp, nxt);
    }
    // backward z hop of this plane (into the next one's accumulator), then
    // the store; the fused dots take the values of q rounded to the storage
    // type.  In the smoother step x += omega r for this plane goes with the
    // store: its x loads are issued before the hop, so the hop's arithmetic
    // covers their latency (updating x when the plane is staged exposes the
    // whole load latency before the barrier).
    S xr[12];
    if (MR) {
      const uint32_t vx = (s * nrhs + r) * IO::SB;
#pragma unroll
      for (int k = 0; k < 12; k++) xr[k] = IO::raw(rx, vx, (uint32_t)k * spb);
    }
    {
      cx<R> gg[2][3];
      {
        S pv[12];
#pragma unroll
        for (int k = 0; k < 12; k++) pv[k] = cur[lidx(k, yl + 1, col)];
        hop_raw<P, PK>(pv, 2, false, ru, upb, s * IO::SB, gg);
      }
      const uint32_t vo = (s * nrhs + r) * IO::SB;
      cx<R> sqr = {0, 0};  // this site's dots in the working precision,
      R sqq = 0;           // accumulated over the march in FP64
#pragma unroll
      for (int k = 0; k < 12; k++) {
        const cx<R> pvk = IO::cvt(cur[lidx(k, yl + 1, col)]);  // centre, re-read from LDS
        if (MR) {
          // r - omega q, and x + omega r
          cx<R> rn = pvk;
          rn.re = fmar(-om.re, acc[k].re, rn.re);
          rn.re = fmar(om.im, acc[k].im, rn.re);
          rn.im = fmar(-om.re, acc[k].im, rn.im);
          rn.im = fmar(-om.im, acc[k].re, rn.im);
          IO::st(rout, vo, (uint32_t)k * spb, rn);
          cx<R> xv = IO::cvt(xr[k]);
          fma_(xv, om, pvk);
          IO::st(rx, vo, (uint32_t)k * spb, xv);
        } else {
          IO::st(rout, vo, (uint32_t)k * spb, acc[k]);
        }
        if (DOT) {
          // q as stored (rounded to the storage type); in the smoother step q
          // is not stored and enters unrounded
          cx<R> os = acc[k];
          if (!MR) {
            S st_;
            P::st(&st_, 0, acc[k]);
            os = P::ld(&st_, 0);
          }
          fmac_(sqr, os, pvk);
          sqq += os.re * os.re + os.im * os.im;
        }
      }
      if (DOT) {
        dqr.re += (double)sqr.re;
        dqr.im += (double)sqr.im;
        dqq += (double)sqq;
      }
#pragma unroll
      for (int k = 0; k < 12; k++) acc[k] = {0, 0};
      hop_add<P>(2, false, (R)-0.5, gg, acc);
    }
    if (kTEarly && i + 1 < zs) t_hops(zp, acc);
  }
  if (DOT) {
    // per-rhs block sums: lane % nbr is the rhs within the group (nbr divides
    // 64); the LDS planes are free after this barrier.  Columns of the other
    // groups' rhs get zeros.
    __syncthreads();
    for (int off = 32; off >= nbr; off >>= 1) {
      dqr.re += __shfl_xor(dqr.re, off, 64);
      dqr.im += __shfl_xor(dqr.im, off, 64);
      dqq += __shfl_xor(dqq, off, 64);
    }
    double2* sw_qr = reinterpret_cast<double2*>(march_smem);  // [16][64]
    double* sw_qq = reinterpret_cast<double*>(march_smem + 16 * 64 * sizeof(double2));
    const int w = tid >> 6, lane = tid & 63;
    if (lane < nbr) {
      sw_qr[w * 64 + lane] = make_double2(dqr.re, dqr.im);
      sw_qq[w * 64 + lane] = dqq;
    }
    __syncthreads();
    if (tid < nrhs) {
      double a = 0, b = 0, n2 = 0;
      if (tid >= rb0 && tid < rb0 + nbr) {
        for (int ww = 0; ww < (int)(blockDim.x >> 6); ww++) {
          a += sw_qr[ww * 64 + tid - rb0].x;
          b += sw_qr[ww * 64 + tid - rb0].y;
          n2 += sw_qq[ww * 64 + tid - rb0];
        }
      }
      dpart[(int64_t)tid * nblocks + blockIdx.x] = make_double2(a, b);
      dpart[(int64_t)(nrhs + tid) * nblocks + blockIdx.x] = make_double2(n2, 0.0);
    }
  }
}

// ------------------------------------------------------------------ host

void FineOp::layout(Arena& a, const Geom& g, FineOp* op) {
  const int64_t V = g.V;
  op->g = g;
  op->U64 = a.take_n<double2>(36 * V);
  op->U32 = a.take_n<float2>(36 * V);
  op->U16 = a.take_n<__half2>(36 * V);
  op->C64 = a.take_n<double>(72 * V);
  op->C32 = a.take_n<float>(72 * V);
  op->C16 = a.take_n<__half>(72 * V);
}

void FineOp::build(const double* gauge_host) {
  once_per_device([] {
    double sig[6][2][2][2][2];
    host_sigma(sig);
    MGM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_sigma), sig, sizeof(sig)));
  });
  const int64_t V = g.V;
  // host [V][4][3][3] complex -> device [mu][9][V]
  std::vector<double2> tmp((size_t)36 * V);
  for (int64_t s = 0; s < V; s++)
    for (int k = 0; k < 36; k++) {
      const double* p = gauge_host + 2 * (s * 36 + k);
      tmp[(size_t)k * V + s] = make_double2(p[0], p[1]);
    }
  MGM_HIP(hipMemcpyAsync(U64, tmp.data(), tmp.size() * sizeof(double2), hipMemcpyHostToDevice,
                         ctx->stream));
  hipLaunchKernelGGL(k_clover, dim3(nblocks_for(V, 128)), dim3(128), 0, ctx->stream, C64, U64, g, m0,
                     csw);
  MGM_LAUNCH_CHECK();
  const int64_t nu = 36 * V, nc = 72 * V;
  hipLaunchKernelGGL(k_cvt_c64_c32, dim3(nblocks_for(nu, 256)), dim3(256), 0, ctx->stream, U32, U64, nu);
  hipLaunchKernelGGL(k_cvt_c64_c16, dim3(nblocks_for(nu, 256)), dim3(256), 0, ctx->stream, U16, U64, nu);
  hipLaunchKernelGGL(k_cvt_r64_r32, dim3(nblocks_for(nc, 256)), dim3(256), 0, ctx->stream, C32, C64, nc);
  hipLaunchKernelGGL(k_cvt_r64_r16, dim3(nblocks_for(nc, 256)), dim3(256), 0, ctx->stream, C16, C64, nc);
  MGM_LAUNCH_CHECK();
  ctx->sync();  // tmp must outlive the copy
}

double FineOp::bytes(mgm_prec p, int nrhs) const {
  double wc = (double)prec_bytes(p), wr = wc / 2;
  return (double)g.V * (36 * wc + 72 * wr + 24.0 * wc * nrhs);
}

// right-hand sides per thread: two for FP32/FP16 with an even count; the
// reducing variant keeps one (with two, its FP64 accumulators and LDS cost
// more occupancy than the shared loads save: measured slower for both)
static int rb_of(mgm_prec p, int nrhs, bool dot) {
  return (!dot && p != MGM_PREC_F64 && nrhs % 2 == 0) ? 2 : 1;
}

int64_t FineOp::nblocks(mgm_prec p, int nrhs, bool dot) const {
  return (g.V * (nrhs / rb_of(p, nrhs, dot)) + 255) / 256;
}

template <bool DOT, int RB>
static void launch_rb(const FineOp& op, mgm_prec p, const void* x, void* y, int nrhs, double2* dpart,
                      bool allow_slab) {
  const Geom& g = op.g;
  const int threads = 256;
  const int64_t nb = (g.V * (nrhs / RB) + 255) / 256;
  // slab mapping needs whole 64-thread chunks per slice and kSlab | T; it
  // then covers exactly nb * 256 = V * nrhs / RB threads
  const int64_t per_slice = (g.V / g.T) * (nrhs / RB);
  const int slab = (allow_slab && per_slice % 64 == 0 && g.T % kSlab == 0 && threads == 64 * kSlab) ? 1 : 0;
  hipStream_t st = op.ctx->stream;
  switch (p) {
    case MGM_PREC_F64:
      MGM_CHECK(RB == 1, MGM_ERR_INVALID_ARG, "FP64 dslash takes one rhs per thread");
      hipLaunchKernelGGL((k_dslash<F64, DOT>), dim3((unsigned)nb), dim3(threads), 0, st, (double2*)y,
                         (const double2*)x, op.U64, op.C64, g, nrhs, nb, slab, dpart);
      break;
    case MGM_PREC_F32:
      if (RB == 2)
        hipLaunchKernelGGL((k_dslash_rb<F32, DOT, 2>), dim3((unsigned)nb), dim3(threads), 0, st, (float2*)y,
                           (const float2*)x, op.U32, op.C32, g, nrhs, nb, slab, dpart);
      else
        hipLaunchKernelGGL((k_dslash<F32, DOT>), dim3((unsigned)nb), dim3(threads), 0, st, (float2*)y,
                           (const float2*)x, op.U32, op.C32, g, nrhs, nb, slab, dpart);
      break;
    case MGM_PREC_F16:
      if (RB == 2)
        hipLaunchKernelGGL((k_dslash_rb<F16, DOT, 2>), dim3((unsigned)nb), dim3(threads), 0, st, (__half2*)y,
                           (const __half2*)x, op.U16, op.C16, g, nrhs, nb, slab, dpart);
      else
        hipLaunchKernelGGL((k_dslash<F16, DOT>), dim3((unsigned)nb), dim3(threads), 0, st, (__half2*)y,
                           (const __half2*)x, op.U16, op.C16, g, nrhs, nb, slab, dpart);
      break;
    default:
      throw Error(MGM_ERR_INVALID_ARG, "dslash precision must be F64, F32 or F16");
  }
  MGM_LAUNCH_CHECK();
}

// Plane-marching shapes (rows per tile, z-planes per block, rhs per block),
// tried in this order.  A shape applies when the tile's thread count
// X * TY * nbr is a multiple of 64 and at most 1024, TY divides Y, zs divides
// Z, nbr divides nrhs and 64, the arrays stay below 4 GiB and the LDS it needs
// fits the device; FP64 keeps the site-parallel kernels (its registers would
// not fit 1024-thread blocks).
struct MarchShape {
  int ty, zs, nbr;
};
static const MarchShape kMarchShapes[] = {
    {4, 16, 8}, {4, 8, 8},  {8, 16, 4},  {8, 8, 4}, {16, 16, 2}, {16, 8, 2}, {8, 8, 2},
    {4, 8, 4},  {4, 8, 2},  {16, 16, 1}, {16, 8, 1}, {8, 8, 1},  {4, 8, 1},  {2, 8, 8},
    {4, 32, 8}, {8, 32, 4}, {4, 32, 4}, {16, 32, 2}};

static size_t march_lds(const Geom& g, mgm_prec p, const MarchShape& m, bool dot) {
  size_t b = (size_t)2 * 12 * (m.ty + 2) * g.X * m.nbr * prec_bytes(p);  // two plane buffers
  if (dot) b = std::max(b, (size_t)16 * 64 * (sizeof(double2) + sizeof(double)));
  return b;
}

static bool march_ok(const FineOp& op, mgm_prec p, int nrhs, const MarchShape& m, bool dot) {
  const Geom& g = op.g;
  if (p != MGM_PREC_F32 && p != MGM_PREC_F16) return false;
  if (m.nbr > nrhs || nrhs % m.nbr != 0 || 64 % m.nbr != 0) return false;
  const int64_t th = (int64_t)g.X * m.ty * m.nbr;
  if (th % 64 != 0 || th > 1024) return false;
  if (g.Y % m.ty != 0 || g.Z % m.zs != 0) return false;
  const double lim = 4294967295.0, cb = (double)prec_bytes(p);
  if (12.0 * g.V * nrhs * cb > lim || 36.0 * g.V * cb > lim || 72.0 * g.V * cb / 2 > lim) return false;
  return march_lds(g, p, m, dot) <= op.ctx->max_lds;
}

// Extra arrays of the smoother-step mode (all null otherwise).
struct MrArgs {
  void* x = nullptr;
  const double2* qr = nullptr;
  const double* qq = nullptr;
};

template <class P, bool DOT, bool MR, int TY, bool PK = false>
static void launch_march_p(const FineOp& op, const typename P::S* U, const typename P::RS* C, const void* x,
                           void* y, int nrhs, const MarchShape& m, int64_t nb, int threads, size_t lds,
                           double2* dpart, const MrArgs& mr) {
  using S = typename P::S;
  auto* k = k_dslash_march<P, DOT, MR, TY, 1024, PK>;
  if (lds > 65536)
    MGM_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k, dim3((unsigned)nb), dim3(threads), lds, op.ctx->stream, (S*)y, (const S*)x, U, C, op.g,
                     nrhs, m.nbr, m.zs, nb, dpart, (S*)mr.x, mr.qr, mr.qq);
  MGM_LAUNCH_CHECK();
}

// Returns the number of blocks (partial-sum columns of the reducing variant).
template <bool DOT, bool MR>
static int64_t launch_march(const FineOp& op, mgm_prec p, const void* x, void* y, int nrhs, double2* dpart,
                            const MarchShape& m, const MrArgs& mr = MrArgs(), bool pk = false) {
  const Geom& g = op.g;
  const int threads = g.X * m.ty * m.nbr;
  const int64_t nb = (int64_t)(nrhs / m.nbr) * g.T * (g.Y / m.ty) * (g.Z / m.zs);
  const size_t lds = march_lds(g, p, m, DOT);
#define MGM_MARCH_TY(PT, UU, CC, PKV)                                                                           \
  switch (m.ty) {                                                                                               \
    case 2: launch_march_p<PT, DOT, MR, 2, PKV>(op, UU, CC, x, y, nrhs, m, nb, threads, lds, dpart, mr); break;   \
    case 4: launch_march_p<PT, DOT, MR, 4, PKV>(op, UU, CC, x, y, nrhs, m, nb, threads, lds, dpart, mr); break;   \
    case 8: launch_march_p<PT, DOT, MR, 8, PKV>(op, UU, CC, x, y, nrhs, m, nb, threads, lds, dpart, mr); break;   \
    case 16: launch_march_p<PT, DOT, MR, 16, PKV>(op, UU, CC, x, y, nrhs, m, nb, threads, lds, dpart, mr); break; \
    default: throw Error(MGM_ERR_SHAPE, "unsupported plane-marching tile");                                     \
  }
  if constexpr (MR) {
    MGM_CHECK(p == MGM_PREC_F16, MGM_ERR_INVALID_ARG, "the fused smoother step runs in FP16 storage");
    if (pk) {
      MGM_MARCH_TY(F16, op.U16, op.C16, true)
    } else {
      MGM_MARCH_TY(F16, op.U16, op.C16, false)
    }
  } else {
    if (p == MGM_PREC_F32) {
      MGM_MARCH_TY(F32, op.U32, op.C32, false)
    } else {
      MGM_MARCH_TY(F16, op.U16, op.C16, false)
    }
  }
#undef MGM_MARCH_TY
  return nb;
}

// Tuned launch shapes.  Site-parallel variants first: 0 (rb_of, slab
// order), 1 the plain block order, and the non-reducing FP32/FP16 kernels
// with an even rhs count also try the other rhs-per-thread count (2, 3);
// then every plane-marching shape that applies.  Untuned, FP16 takes the
// first plane-marching shape that applies (measured fastest for the fused
// smoother's 8 and 4 rhs on 32^3 x 64), FP32 and FP64 variant 0.  Returns the
// block count of the variant that ran.
template <bool DOT>
static int64_t launch_dslash(const FineOp& op, mgm_prec p, const void* x, void* y, int nrhs, double2* dpart) {
  const int rb0 = rb_of(p, nrhs, DOT);
  const bool alt = !DOT && p != MGM_PREC_F64 && nrhs % 2 == 0;
  const int nsite = alt ? 4 : 2;
  std::vector<MarchShape> shapes;
  for (const MarchShape& m : kMarchShapes)
    if (march_ok(op, p, nrhs, m, DOT)) shapes.push_back(m);
  const std::string key = std::string(DOT ? "dslash_dot/" : "dslash/") + std::to_string((int)p) + "/" +
                          std::to_string(op.g.V) + "/" + std::to_string(nrhs);
  int64_t nb = 0;
  const int dflt = (p == MGM_PREC_F16 && !shapes.empty()) ? nsite : 0;
  op.ctx->choose(
      key, nsite + (int)shapes.size(),
      [&](int v) {
    MGM_CHECK(v >= 0 && v < nsite + (int)shapes.size(), MGM_ERR_INVALID_ARG,
              "dslash launch variant out of range for this shape");
    if (v >= nsite) {
      nb = launch_march<DOT, false>(op, p, x, y, nrhs, dpart, shapes[v - nsite]);
      return;
    }
    const int rb = v < 2 ? rb0 : 3 - rb0;
    const bool slab = (v & 1) == 0;
    if (rb == 2)
      launch_rb<DOT, 2>(op, p, x, y, nrhs, dpart, slab);
    else
      launch_rb<DOT, 1>(op, p, x, y, nrhs, dpart, slab);
    nb = (op.g.V * (nrhs / rb) + 255) / 256;
      },
      dflt);
  return nb;
}

static int kclass_of(mgm_prec p) {
  return p == MGM_PREC_F64 ? KC_DSLASH_F64 : p == MGM_PREC_F32 ? KC_DSLASH_F32 : KC_DSLASH_F16;
}

void FineOp::apply(mgm_prec p, const void* x, void* y, int nrhs) const {
  ProfScope ps(ctx, kclass_of(p), bytes(p, nrhs));
  launch_dslash<false>(*this, p, x, y, nrhs, nullptr);
}

int64_t FineOp::apply_dot(mgm_prec p, const void* x, void* y, int nrhs, double2* dpart) const {
  // one block holds 256 elements; each rhs needs a reducing thread
  MGM_CHECK(nrhs >= 1 && nrhs <= 256, MGM_ERR_INVALID_ARG, "fused dslash reduction supports 1..256 rhs");
  ProfScope ps(ctx, kclass_of(p), bytes(p, nrhs));
  return launch_dslash<true>(*this, p, x, y, nrhs, dpart);
}

bool FineOp::step_fusable(mgm_prec p, int nrhs) const {
  if (p != MGM_PREC_F16) return false;
  for (const MarchShape& m : kMarchShapes)
    if (march_ok(*this, p, nrhs, m, true)) return true;
  return false;
}

double FineOp::step_bytes(mgm_prec p, int nrhs) const {
  // the dslash (r in, r' out in place of q), plus x read and written
  return bytes(p, nrhs) + 2.0 * 12.0 * (double)g.V * nrhs * (double)prec_bytes(p);
}

int64_t FineOp::apply_step(mgm_prec p, const void* r, void* r_next, void* x, const double2* qr, const double* qq,
                           int nrhs, double2* dpart) const {
  MGM_CHECK(step_fusable(p, nrhs), MGM_ERR_SHAPE, "no plane-marching tile for the fused smoother step");
  MGM_CHECK(r != r_next && r != x && r_next != x, MGM_ERR_INVALID_ARG, "fused smoother step needs distinct arrays");
  std::vector<MarchShape> shapes;
  for (const MarchShape& m : kMarchShapes)
    if (march_ok(*this, p, nrhs, m, true)) shapes.push_back(m);
  MrArgs mr;
  mr.x = x;
  mr.qr = qr;
  mr.qq = qq;
  const std::string key = "dslash_step/" + std::to_string((int)p) + "/" + std::to_string(g.V) + "/" + std::to_string(nrhs);
  ProfScope ps(ctx, KC_DSLASH_STEP, step_bytes(p, nrhs));
  int64_t nb = 0;
  // variants: every shape with FP32 arithmetic on converted values, then
  // every shape with packed FP16 arithmetic
  const int ns = (int)shapes.size();
  ctx->choose(key, 2 * ns, [&](int v) {
    MGM_CHECK(v >= 0 && v < 2 * ns, MGM_ERR_INVALID_ARG, "fused smoother launch variant out of range");
    nb = launch_march<true, true>(*this, p, r, r_next, nrhs, dpart, shapes[v % ns], mr, v >= ns);
  });
  return nb;
}

}  // namespace mgm
