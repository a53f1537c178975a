// Learned gauge-covariant smoother: parallel-transport convolution (PTC)
// layers out_a = sum_p W_p[a][b] T_p in_b over the identity and the eight
// nearest-neighbour transports, their weight and input gradients, full-batch
// Adam, and the training-pair generation from multigrid solves.
//
// Layout: channel-major like the fine spinors, element
// ((channel * 3 + colour) * V + site) * nrhs + rhs, FP32 complex.  A thread
// handles one (site, rhs) and all output channels of a layer; the weights are
// uniform across the wave and come through the scalar cache.
#include "net.h"

#include <chrono>
#include <cmath>
#include <random>

namespace mgm {

// ------------------------------------------------------------ transports

// (T_p in_b)(s) for the three colours of channel b.  p = 0 identity,
// 1 + mu: U_mu(s) in(s + mu); 5 + mu: U_mu(s - mu)^H in(s - mu); the hop
// across the time boundary carries the antiperiodic sign.
__device__ __forceinline__ void ptc_transport(const float2* __restrict__ in, const float2* __restrict__ U,
                                              const Geom& g, int64_t s, const int c[4], int p, int b,
                                              int nrhs, int r, cx<float> t[3]) {
  const int64_t V = g.V;
  if (p == 0) {
#pragma unroll
    for (int cc = 0; cc < 3; cc++) {
      float2 v = in[((int64_t)(b * 3 + cc) * V + s) * nrhs + r];
      t[cc] = {v.x, v.y};
    }
    return;
  }
  const int mu = (p - 1) & 3;
  const bool fwd = p <= 4;
  const int cm = c[mu];
  const int ex = mu == 0 ? g.X : mu == 1 ? g.Y : mu == 2 ? g.Z : g.T;
  const int64_t sd = mu == 0 ? 1 : mu == 1 ? (int64_t)g.X : mu == 2 ? (int64_t)g.X * g.Y
                                                                     : (int64_t)g.X * g.Y * g.Z;
  const bool wrap = fwd ? (cm == ex - 1) : (cm == 0);
  const int64_t span = (int64_t)(ex - 1) * sd;
  const int64_t sn = fwd ? (wrap ? s - span : s + sd) : (wrap ? s + span : s - sd);
  const float ph = (mu == 3 && wrap && g.antiperiodic) ? -1.f : 1.f;
  cx<float> v[3];
#pragma unroll
  for (int cc = 0; cc < 3; cc++) {
    float2 w = in[((int64_t)(b * 3 + cc) * V + sn) * nrhs + r];
    v[cc] = {ph * w.x, ph * w.y};
  }
  const float2* Ub = U + (int64_t)(mu * 9) * V + (fwd ? s : sn);
#pragma unroll
  for (int a = 0; a < 3; a++) {
    cx<float> acc = {0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 3; k++) {
      if (fwd) {
        float2 u = Ub[(int64_t)(3 * a + k) * V];
        fma_(acc, cx<float>{u.x, u.y}, v[k]);
      } else {
        float2 u = Ub[(int64_t)(3 * k + a) * V];  // (U^H)_{ak} = conj(U_{ka})
        fmac_(acc, cx<float>{u.x, u.y}, v[k]);
      }
    }
    t[a] = acc;
  }
}

__device__ __forceinline__ void site_coords(const Geom& g, int64_t s, int c[4]) {
  int64_t q = s;
  c[0] = (int)(q % g.X);
  q /= g.X;
  c[1] = (int)(q % g.Y);
  q /= g.Y;
  c[2] = (int)(q % g.Z);
  c[3] = (int)(q / g.Z);
}

// out = sum_p W_p T_p in ; W [9][CO][ci]
template <int CO>
__global__ __launch_bounds__(256) void k_ptc_layer(float2* __restrict__ out, const float2* __restrict__ in,
                                                   const float2* __restrict__ U, const float2* __restrict__ W,
                                                   Geom g, int ci, int nrhs) {
  const int64_t V = g.V, N = V * nrhs;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= N) return;
  const int64_t s = tid / nrhs;
  const int r = (int)(tid - s * nrhs);
  int c[4];
  site_coords(g, s, c);
  cx<float> acc[CO][3];
#pragma unroll
  for (int a = 0; a < CO; a++)
#pragma unroll
    for (int cc = 0; cc < 3; cc++) acc[a][cc] = {0.f, 0.f};
#pragma unroll 1
  for (int p = 0; p < kNetPaths; p++) {
    const float2* Wp = W + (int64_t)p * CO * ci;
#pragma unroll 1
    for (int b = 0; b < ci; b++) {
      cx<float> t[3];
      ptc_transport(in, U, g, s, c, p, b, nrhs, r, t);
#pragma unroll
      for (int a = 0; a < CO; a++) {
        const float2 wv = Wp[a * ci + b];
        const cx<float> w = {wv.x, wv.y};
#pragma unroll
        for (int cc = 0; cc < 3; cc++) fma_(acc[a][cc], w, t[cc]);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < CO; a++)
#pragma unroll
    for (int cc = 0; cc < 3; cc++)
      out[((int64_t)(a * 3 + cc) * V + s) * nrhs + r] = make_float2(acc[a][cc].re, acc[a][cc].im);
}

// Weight gradient of one layer: part[blk][p][a][b] = sum over the block's
// elements of gout_a conj(T_p in_b), summed over colours (grid nblk x 9).
constexpr int kWE = 32;  // elements staged per tile
__global__ __launch_bounds__(256) void k_ptc_wgrad(const float2* __restrict__ gout, const float2* __restrict__ in,
                                                   const float2* __restrict__ U, Geom g, int co, int ci, int nrhs,
                                                   int64_t per_block, double2* __restrict__ part) {
  const int p = blockIdx.y;
  const int64_t V = g.V, N = V * nrhs;
  const int64_t e0 = (int64_t)blockIdx.x * per_block;
  const int64_t e1 = e0 + per_block < N ? e0 + per_block : N;
  __shared__ float2 sG[kNetMaxWidth * 3][kWE];
  __shared__ float2 sX[kNetMaxWidth * 3][kWE];
  const int t = threadIdx.x;
  const bool pair = t < co * ci;
  const int a = pair ? t / ci : 0, b = pair ? t % ci : 0;
  double ar = 0, ai = 0;
  for (int64_t eb = e0; eb < e1; eb += kWE) {
    for (int j = t; j < co * 3 * kWE; j += blockDim.x) {
      const int ac = j / kWE, e = j % kWE;
      const int64_t el = eb + e;
      sG[ac][e] = el < e1 ? gout[(int64_t)ac * N + el] : make_float2(0.f, 0.f);
    }
    for (int j = t; j < ci * kWE; j += blockDim.x) {
      const int bb = j / kWE, e = j % kWE;
      const int64_t el = eb + e;
      cx<float> tt[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
      if (el < e1) {
        const int64_t s = el / nrhs;
        const int r = (int)(el - s * nrhs);
        int c[4];
        site_coords(g, s, c);
        ptc_transport(in, U, g, s, c, p, bb, nrhs, r, tt);
      }
#pragma unroll
      for (int cc = 0; cc < 3; cc++) sX[bb * 3 + cc][e] = make_float2(tt[cc].re, tt[cc].im);
    }
    __syncthreads();
    if (pair) {
      float fr = 0.f, fi = 0.f;
      for (int e = 0; e < kWE; e++)
#pragma unroll
        for (int cc = 0; cc < 3; cc++) {
          const float2 gv = sG[a * 3 + cc][e], xv = sX[b * 3 + cc][e];
          fr += gv.x * xv.x + gv.y * xv.y;  // g conj(x)
          fi += gv.y * xv.x - gv.x * xv.y;
        }
      ar += fr;
      ai += fi;
    }
    __syncthreads();
  }
  if (pair) part[((int64_t)blockIdx.x * kNetPaths + p) * co * ci + t] = make_double2(ar, ai);
}

// out[i] = sum_blk part[blk][i], one 64-lane wave per entry, fixed order
__global__ void k_ptc_wsum(const double2* __restrict__ part, int64_t nblk, int cnt, double2* __restrict__ out) {
  const int i = blockIdx.x;
  double a = 0, b = 0;
  for (int64_t k = threadIdx.x; k < nblk; k += 64) {
    const double2 v = part[k * cnt + i];
    a += v.x;
    b += v.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  if (threadIdx.x == 0) out[i] = make_double2(a, b);
}

// FP32 forward weights and backward weights W'_q = W_{opposite(q)}^H
// FP32 value rounded to the nearest BF16 value (ties to even), kept in FP32
__device__ __forceinline__ float round_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// kernel weights from the master weights: FP32, or BF16-rounded when bf16
// (the layers then multiply BF16 weights and accumulate in FP32)
__global__ void k_ptc_wcopy(const double2* __restrict__ w64, float2* __restrict__ w32, float2* __restrict__ wadj,
                            int co, int ci, int bf16) {
  const int n = kNetPaths * co * ci;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int p = i / (co * ci), rem = i % (co * ci), a = rem / ci, b = rem % ci;
    const double2 w = w64[i];
    float wr = (float)w.x, wi = (float)w.y;
    if (bf16) {
      wr = round_bf16(wr);
      wi = round_bf16(wi);
    }
    w32[i] = make_float2(wr, wi);
    const int q = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
    wadj[(q * ci + b) * co + a] = make_float2(wr, -wi);
  }
}

// Adam on real and imaginary parts as separate parameters
__global__ void k_ptc_adam(double2* __restrict__ w, const double2* __restrict__ g, double2* __restrict__ m,
                           double2* __restrict__ v, int64_t n, double lr, double b1, double b2, double eps,
                           double c1, double c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double2 gi = g[i];
    double2 mi = m[i], vi = v[i], wi = w[i];
    mi.x = b1 * mi.x + (1 - b1) * gi.x;
    mi.y = b1 * mi.y + (1 - b1) * gi.y;
    vi.x = b2 * vi.x + (1 - b2) * gi.x * gi.x;
    vi.y = b2 * vi.y + (1 - b2) * gi.y * gi.y;
    wi.x -= lr * (mi.x / c1) / (sqrt(vi.x / c2) + eps);
    wi.y -= lr * (mi.y / c1) / (sqrt(vi.y / c2) + eps);
    m[i] = mi;
    v[i] = vi;
    w[i] = wi;
  }
}

// loss = mean_j n2_j / e2_j and the per-rhs output-gradient scale 2 / (n e2_j)
__global__ void k_ptc_loss(const double* n2, const double* e2, int nrhs, double* scale, double* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double l = 0;
  for (int j = 0; j < nrhs; j++) {
    const double d = e2[j];
    l += d > 0 ? n2[j] / d : 0.0;
    scale[j] = d > 0 ? 2.0 / (nrhs * d) : 0.0;
  }
  *loss = l / nrhs;
}

// ------------------------------------------------------------------ host

static void launch_layer(Context* c, const FineOp* op, float2* out, const float2* in, const float2* W, int co,
                         int ci, int nrhs) {
  const int64_t N = op->g.V * nrhs;
  const dim3 nb(nblocks_for(N, 256)), tb(256);
  ProfScope ps(c, KC_NET, (double)op->g.V * (36.0 * 8 + (co + 9.0 * ci) * 3 * 8 * nrhs));
  switch (co) {
    case 4: hipLaunchKernelGGL(k_ptc_layer<4>, nb, tb, 0, c->stream, out, in, op->U32, W, op->g, ci, nrhs); break;
    case 8: hipLaunchKernelGGL(k_ptc_layer<8>, nb, tb, 0, c->stream, out, in, op->U32, W, op->g, ci, nrhs); break;
    case 12: hipLaunchKernelGGL(k_ptc_layer<12>, nb, tb, 0, c->stream, out, in, op->U32, W, op->g, ci, nrhs); break;
    case 16: hipLaunchKernelGGL(k_ptc_layer<16>, nb, tb, 0, c->stream, out, in, op->U32, W, op->g, ci, nrhs); break;
    default: throw Error(MGM_ERR_INVALID_ARG, "network widths must be 4, 8, 12 or 16");
  }
  MGM_LAUNCH_CHECK();
}

static int64_t wgrad_blocks(int64_t N) {
  int64_t nb = (N + 2047) / 2048;
  return nb < 1 ? 1 : (nb > 512 ? 512 : nb);
}

void Net::layout(Arena& a) {
  L = desc.nlayers;
  nw = 0;
  int wmax = 4, whid = 4;
  for (int l = 0; l <= L; l++) {
    width[l] = desc.width[l];
    wmax = std::max(wmax, width[l]);
    if (l > 0 && l < L) whid = std::max(whid, width[l]);
  }
  for (int l = 0; l < L; l++) {
    woff[l] = nw;
    nw += (int64_t)kNetPaths * width[l + 1] * width[l];
  }
  woff[L] = nw;
  w64 = a.take_n<double2>(nw);
  g64 = a.take_n<double2>(nw);
  m = a.take_n<double2>(nw);
  v = a.take_n<double2>(nw);
  w32 = a.take_n<float2>(nw);
  wadj = a.take_n<float2>(nw);
  const int64_t V = op->g.V;
  const int64_t na = (int64_t)whid * 3 * V * desc.max_nrhs;
  buf[0] = a.take_n<float2>(na);
  buf[1] = a.take_n<float2>(na);
  const int B = desc.train_nrhs;
  if (B > 0) {
    for (int l = 0; l <= L; l++) act[l] = a.take_n<float2>((size_t)width[l] * 3 * V * B);
    gbuf[0] = a.take_n<float2>((size_t)wmax * 3 * V * B);
    gbuf[1] = a.take_n<float2>((size_t)wmax * 3 * V * B);
    tr_e = a.take_n<float2>((size_t)12 * V * B);
    wpart_blocks = wgrad_blocks(V * B);
    wpart = a.take_n<double2>((size_t)wpart_blocks * kNetPaths * kNetMaxWidth * kNetMaxWidth);
    n2 = a.take_n<double>(B);
    e2 = a.take_n<double>(B);
    scale = a.take_n<double>(B);
    loss = a.take_n<double>(1);
    scratch.cap = (size_t)kRedBlocksMax * B;
    scratch.partial = a.take_n<double2>(scratch.cap);
  }
}

void Net::refresh() {
  for (int l = 0; l < L; l++) {
    const int co = width[l + 1], ci = width[l];
    hipLaunchKernelGGL(k_ptc_wcopy, dim3(nblocks_for((int64_t)kNetPaths * co * ci, 256)), dim3(256), 0,
                       ctx->stream, w64 + woff[l], w32 + woff[l], wadj + woff[l], co, ci, desc.bf16_weights ? 1 : 0);
  }
  MGM_LAUNCH_CHECK();
}

void Net::upload_weights(const std::vector<double>& host) {
  MGM_CHECK((int64_t)host.size() == 2 * nw, MGM_ERR_INVALID_ARG, "weight count mismatch");
  MGM_HIP(hipMemcpyAsync(w64, host.data(), sizeof(double2) * nw, hipMemcpyHostToDevice, ctx->stream));
  MGM_HIP(hipMemsetAsync(m, 0, sizeof(double2) * nw, ctx->stream));
  MGM_HIP(hipMemsetAsync(v, 0, sizeof(double2) * nw, ctx->stream));
  adam_step = 0;
  refresh();
  ctx->sync();  // host vector must outlive the copy
}

void Net::apply(const float2* r, float2* y, int nrhs) {
  MGM_CHECK(nrhs >= 1 && nrhs <= desc.max_nrhs, MGM_ERR_INVALID_ARG, "nrhs exceeds the network's max_nrhs");
  for (int l = 0; l < L; l++) {
    const float2* in = l == 0 ? r : buf[(l - 1) & 1];
    float2* out = l == L - 1 ? y : buf[l & 1];
    launch_layer(ctx, op, out, in, w32 + woff[l], width[l + 1], width[l], nrhs);
  }
}

double Net::loss_grad(const float2* r, const float2* e, int nrhs) {
  MGM_CHECK(desc.train_nrhs > 0 && nrhs >= 1 && nrhs <= desc.train_nrhs, MGM_ERR_INVALID_ARG,
            "nrhs exceeds the network's train_nrhs");
  Context* c = ctx;
  const int64_t V = op->g.V, N = V * nrhs;
  auto in_of = [&](int l) { return l == 0 ? r : (const float2*)act[l]; };
  for (int l = 0; l < L; l++) launch_layer(c, op, act[l + 1], in_of(l), w32 + woff[l], width[l + 1], width[l], nrhs);
  // output gradient 2 (N(r) - e) / (n |e|^2), in place of the output
  Vec od;
  od.p = act[L];
  od.nsite = V;
  od.dof = 12;
  od.nrhs = nrhs;
  od.prec = MGM_PREC_F32;
  Vec ev = od.with((void*)e);
  b_axpy(c, nullptr, -1.0, ev, od);
  b_norm2(c, scratch, od, n2);
  b_norm2(c, scratch, ev, e2);
  hipLaunchKernelGGL(k_ptc_loss, dim3(1), dim3(1), 0, c->stream, n2, e2, nrhs, scale, loss);
  MGM_LAUNCH_CHECK();
  b_scale_rhs(c, od, scale);
  const float2* G = act[L];
  const int64_t nblk = wgrad_blocks(N);
  const int64_t per = ((N + nblk - 1) / nblk + kWE - 1) / kWE * kWE;
  for (int l = L - 1; l >= 0; l--) {
    const int co = width[l + 1], ci = width[l];
    const int64_t nb = (N + per - 1) / per;
    hipLaunchKernelGGL(k_ptc_wgrad, dim3((unsigned)nb, kNetPaths), dim3(256), 0, c->stream, G, in_of(l), op->U32,
                       op->g, co, ci, nrhs, per, wpart);
    const int cnt = kNetPaths * co * ci;
    hipLaunchKernelGGL(k_ptc_wsum, dim3(cnt), dim3(64), 0, c->stream, wpart, nb, cnt, g64 + woff[l]);
    MGM_LAUNCH_CHECK();
    if (l > 0) {
      float2* Gn = gbuf[l & 1];
      // input gradient: sum_q T_q (W_{opposite q}^H G), a layer with c_out = ci
      launch_layer(c, op, Gn, G, wadj + woff[l], ci, co, nrhs);
      G = Gn;
    }
  }
  MGM_HIP(hipMemcpyAsync(pinned, loss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  return pinned[0];
}

void Net::adam(double lr, double b1, double b2, double eps) {
  adam_step++;
  const double c1 = 1.0 - std::pow(b1, (double)adam_step), c2 = 1.0 - std::pow(b2, (double)adam_step);
  hipLaunchKernelGGL(k_ptc_adam, dim3(nblocks_for(nw, 256)), dim3(256), 0, ctx->stream, w64, g64, m, v, nw, lr, b1,
                     b2, eps, c1, c2);
  MGM_LAUNCH_CHECK();
  refresh();
}

void net_apply(Hier& H, Net& net, Vec r, Vec e) {
  MGM_CHECK(r.prec == MGM_PREC_F32 && e.prec == MGM_PREC_F32, MGM_ERR_INVALID_ARG,
            "the network smoother runs on FP32 vectors (solve kind NET)");
  MGM_CHECK(net.op == H.fine, MGM_ERR_INVALID_ARG, "network and hierarchy belong to different operators");
  net.apply((const float2*)r.p, (float2*)e.p, r.nrhs);
}

void net_train(Hier& H, Net& net, const mgm_train_desc& d, mgm_train_stats* st, double* history) {
  const auto t0 = std::chrono::steady_clock::now();
  const int B = net.desc.train_nrhs;
  MGM_CHECK(B > 0, MGM_ERR_INVALID_ARG, "network was created without training buffers (train_nrhs = 0)");
  MGM_CHECK(net.op == H.fine, MGM_ERR_INVALID_ARG, "network and hierarchy belong to different operators");
  MGM_CHECK(H.L >= 2 && B <= H.cap(0), MGM_ERR_INVALID_ARG, "hierarchy rhs capacity below train_nrhs");
  MGM_CHECK(d.steps >= 1 && d.lr > 0 && d.target_tol > 0, MGM_ERR_INVALID_ARG, "bad training parameters");
  Context* c = H.ctx;
  const int64_t V = H.g[0].V;
  // pairs: z (Z4), e_c = P D_c^-1 P^H z, r = z - D e_c, e = D^-1 r
  double2 *z = H.est.x[0], *ec = H.est.y[0], *rr = H.est.z[0], *ee = H.est.w[0];
  double2 *zc = H.est.x[1], *xc = H.est.y[1];
  draw_z4(c, d.seed, (uint32_t)(256 * 0 + 8), 0, B, V, 12, MGM_PREC_F64, z);
  SolveCfg sc;
  sc.tol = d.target_tol;
  sc.maxiter = 4000;
  sc.kind = MGM_SOLVE_MG;
  sc.smooth = 4;
  sc.coarse_iters = 8;
  MGM_CHECK(H.ws64[0].V != nullptr, MGM_ERR_INVALID_ARG, "training needs FP64 Krylov workspaces (mixed != 1)");
  H.T[0].restrict_(MGM_PREC_F64, z, zc, B);
  SolveOut so1, so0;
  solve(H, 1, sc, zc, xc, B, &so1);
  H.T[0].prolong(MGM_PREC_F64, xc, nullptr, ec, B, 0);
  H.apply(0, MGM_PREC_F64, ec, rr, B);
  Vec zv = H.vec(0, MGM_PREC_F64, z, B);
  b_xpay(c, zv, nullptr, -1.0, zv.with(rr));  // r = z - D e_c
  solve(H, 0, sc, rr, ee, B, &so0);
  MGM_CHECK(so0.converged && so1.converged, MGM_ERR_NOT_CONVERGED, "training-target solves did not converge");
  Vec r32 = H.vec(0, MGM_PREC_F32, net.act[0], B);
  b_copy(c, r32, zv.with(rr));
  b_copy(c, r32.with(net.tr_e), zv.with(ee));
  const double b1 = d.beta1 > 0 ? d.beta1 : 0.9, b2 = d.beta2 > 0 ? d.beta2 : 0.999;
  const double eps = d.eps > 0 ? d.eps : 1e-8;
  double first = 0, last = 0;
  for (int it = 0; it < d.steps; it++) {
    const double l = net.loss_grad(net.act[0], net.tr_e, B);
    MGM_CHECK(std::isfinite(l), MGM_ERR_NUMERIC, "non-finite training loss");
    if (it == 0) first = l;
    last = l;
    if (history) history[it] = l;
    net.adam(d.lr, b1, b2, eps);
  }
  c->sync();
  if (st) {
    st->loss_first = first;
    st->loss_last = last;
    st->steps = d.steps;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
}

// initial weights: identity path with a 1/(4 + m0)-like scale on the first
// layer (the inverse of the Wilson diagonal), identity elsewhere, plus small
// Gaussian noise on every entry
std::vector<double> net_initial_weights(const Net& n, uint64_t seed) {
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> w(2 * n.nw, 0.0);
  for (int l = 0; l < n.L; l++) {
    const int co = n.width[l + 1], ci = n.width[l];
    const double noise = 0.01 / std::sqrt((double)kNetPaths * ci);
    for (int p = 0; p < kNetPaths; p++)
      for (int a = 0; a < co; a++)
        for (int b = 0; b < ci; b++) {
          const int64_t i = n.woff[l] + ((int64_t)p * co + a) * ci + b;
          double re = noise * nd(gen), im = noise * nd(gen);
          if (p == 0 && a == b) re += l == 0 ? 0.25 : 1.0;
          w[2 * i] = re;
          w[2 * i + 1] = im;
        }
  }
  return w;
}

}  // namespace mgm
