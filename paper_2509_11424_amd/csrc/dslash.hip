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
      g0 = f * g0;
      g1 = f * g1;
      cx<R> d0, d1;
      Ad_times(mu, g0, g1, d0, d1);  // lower spins: -A^H g (forward), +A^H g (backward)
      acc[0 * 3 + a] = acc[0 * 3 + a] + g0;
      acc[1 * 3 + a] = acc[1 * 3 + a] + g1;
      acc[2 * 3 + a] = acc[2 * 3 + a] + sg * d0;
      acc[3 * 3 + a] = acc[3 * 3 + a] + sg * d1;
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
        g0 = f * g0;
        g1 = f * g1;
        cx<R> d0, d1;
        Ad_times(mu, g0, g1, d0, d1);  // lower spins: -A^H g (forward), +A^H g (backward)
        acc[0 * 3 + a][j] = acc[0 * 3 + a][j] + g0;
        acc[1 * 3 + a][j] = acc[1 * 3 + a][j] + g1;
        acc[2 * 3 + a][j] = acc[2 * 3 + a][j] + sg * d0;
        acc[3 * 3 + a][j] = acc[3 * 3 + a][j] + sg * d1;
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
  static bool sigma_ready = false;
  if (!sigma_ready) {
    double sig[6][2][2][2][2];
    host_sigma(sig);
    MGM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_sigma), sig, sizeof(sig)));
    sigma_ready = true;
  }
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

// Tuned launch shapes: variant 0 is the default (rb_of, slab order), 1 the
// plain block order; the non-reducing FP32/FP16 kernels with an even rhs count
// also try the other rhs-per-thread count (2, 3).  The reducing variant keeps
// rb_of, whose block count sizes the partial sums.
template <bool DOT>
static void launch_dslash(const FineOp& op, mgm_prec p, const void* x, void* y, int nrhs, double2* dpart) {
  const int rb0 = rb_of(p, nrhs, DOT);
  const bool alt = !DOT && p != MGM_PREC_F64 && nrhs % 2 == 0;
  const std::string key = std::string(DOT ? "dslash_dot/" : "dslash/") + std::to_string((int)p) + "/" +
                          std::to_string(op.g.V) + "/" + std::to_string(nrhs);
  op.ctx->choose(key, alt ? 4 : 2, [&](int v) {
    const int rb = v < 2 ? rb0 : 3 - rb0;
    const bool slab = (v & 1) == 0;
    if (rb == 2)
      launch_rb<DOT, 2>(op, p, x, y, nrhs, dpart, slab);
    else
      launch_rb<DOT, 1>(op, p, x, y, nrhs, dpart, slab);
  });
}

static int kclass_of(mgm_prec p) {
  return p == MGM_PREC_F64 ? KC_DSLASH_F64 : p == MGM_PREC_F32 ? KC_DSLASH_F32 : KC_DSLASH_F16;
}

void FineOp::apply(mgm_prec p, const void* x, void* y, int nrhs) const {
  ProfScope ps(ctx, kclass_of(p), bytes(p, nrhs));
  launch_dslash<false>(*this, p, x, y, nrhs, nullptr);
}

void FineOp::apply_dot(mgm_prec p, const void* x, void* y, int nrhs, double2* dpart) const {
  // one block holds 256 elements; each rhs needs a reducing thread
  MGM_CHECK(nrhs >= 1 && nrhs <= 256, MGM_ERR_INVALID_ARG, "fused dslash reduction supports 1..256 rhs");
  ProfScope ps(ctx, kclass_of(p), bytes(p, nrhs));
  launch_dslash<true>(*this, p, x, y, nrhs, dpart);
}

}  // namespace mgm
