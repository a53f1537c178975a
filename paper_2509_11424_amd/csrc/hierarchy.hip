// Multigrid hierarchy: workspace layout and the adaptive setup (Sec. 2.2:
// aggregation-based unitary P_l from N_tv test vectors approximating low
// modes of D_l, Galerkin D_{l+1} = P_l^H D_l P_l).
#include "lib.h"
#include "block.h"

namespace mgm {

void Hier::apply(int l, mgm_prec p, const void* x, void* y, int nrhs) const {
  if (l == 0)
    fine->apply(p, x, y, nrhs);
  else
    A[l].apply(p, x, y, nrhs);
}

// FP16 fine-level smoother: input, result, MR residual and product vectors
static void carve_smooth16(Arena& a, LevelWS& w, int64_t n, int nmax) {
  w.prec = MGM_PREC_F16;
  w.nmax = nmax;
  const size_t vb = (size_t)n * nmax * prec_bytes(MGM_PREC_F16);
  w.r = a.take(vb);
  w.t = a.take(vb);
  w.rho = a.take(vb);
  w.q = a.take(vb);
  w.n2a = a.take_n<double>(nmax);
  w.n2b = a.take_n<double>(nmax);
  w.qr = a.take_n<double2>(nmax);
  w.qq = a.take_n<double>(nmax);
  w.qr2 = a.take_n<double2>(nmax);
  w.qq2 = a.take_n<double>(nmax);
  w.mask = a.take_n<double>(nmax);
}

static void carve_ws(Arena& a, LevelWS& w, mgm_prec p, int64_t n, int nmax, int m, bool krylov) {
  w.prec = p;
  w.nmax = nmax;
  w.m = m;
  const size_t vb = (size_t)n * nmax * prec_bytes(p);
  if (krylov) {
    w.V = a.take(vb * (m + 1));
    w.Z = a.take(vb * m);
    w.rho = a.take(vb);
    w.q = a.take(vb);
    w.y = a.take(vb);
    w.bc = a.take(vb);
    w.xc = a.take(vb);
  }
  w.r = a.take(vb);
  w.t = a.take(vb);
  const size_t mm = (size_t)m * m * nmax, m1 = (size_t)(m + 1) * nmax;
  w.G.m = m;
  w.G.R = a.take_n<double2>(mm);
  w.G.cs = a.take_n<double>((size_t)m * nmax);
  w.G.sn = a.take_n<double2>((size_t)m * nmax);
  w.G.g = a.take_n<double2>(m1);
  w.G.h = a.take_n<double2>(m1);
  w.G.h2 = a.take_n<double2>(m1);
  w.G.beta = a.take_n<double>(nmax);
  w.G.est = a.take_n<double>(nmax);
  w.G.y = a.take_n<double2>((size_t)m * nmax);
  w.n2a = a.take_n<double>(nmax);
  w.n2b = a.take_n<double>(nmax);
  w.qr = a.take_n<double2>(nmax);
  w.qq = a.take_n<double>(nmax);
  w.mask = a.take_n<double>(nmax);
}

void Hier::layout(Arena& a) {
  L = desc.nlevels;
  g.assign(L, LGeom{});
  T.assign(L > 0 ? L - 1 : 0, Transfer{});
  A.assign(L, CoarseOp{});
  g[0].dims[0] = fine->g.X;
  g[0].dims[1] = fine->g.Y;
  g[0].dims[2] = fine->g.Z;
  g[0].dims[3] = fine->g.T;
  g[0].V = fine->g.V;
  g[0].dof = 12;
  for (int l = 0; l + 1 < L; l++) {
    T[l].ctx = ctx;
    T[l].t = make_tgeom(g[l], desc.block[l], desc.ntv[l]);
    g[l + 1] = T[l].t.c;
    A[l + 1].ctx = ctx;
    A[l + 1].g = g[l + 1];
    A[l + 1].d = g[l + 1].dof;
  }
  const bool mixed = desc.mixed != 0;
  const bool full64 = desc.mixed != 1;
  // persistent objects
  for (int l = 0; l + 1 < L; l++) {
    const TGeom& t = T[l].t;
    size_t np = (size_t)t.c.V * 2 * t.rows * t.ntv;
    T[l].P64 = a.take_n<double2>(np);
    if (mixed) T[l].P16 = a.take_n<__half2>(np);
    CoarseOp& C = A[l + 1];
    size_t na = (size_t)9 * C.d * C.d * C.g.V;
    C.A64 = a.take_n<double2>(na);
    C.Ap64 = (double2*)a.take(mg_mfma64_bytes(C));
    if (mixed) {
      C.A32 = (float2*)a.take(mg_mfma32_bytes(C));
      C.Abf = a.take(mg_mfma_bytes(C));
    }
  }
  d_flag = a.take_n<int>(64);
  int ntv_max = 0;
  for (int l = 0; l + 1 < L; l++) ntv_max = std::max(ntv_max, desc.ntv[l]);
  const int nmax = cap(L - 1), nfine = cap(0);
  const int red_n = std::max(nmax, ntv_max);
  const int m = desc.restart;
  scratch.cap = (size_t)kRedBlocksMax * kFusedGS * red_n;
  scratch.partial = a.take_n<double2>(scratch.cap);
  dpart = a.take_n<double2>((size_t)fine->nblocks(MGM_PREC_F64, nfine, true) * 2 * nfine);
  // estimator buffers (FP64)
  est.nmax = nmax;
  est.x.assign(L, nullptr);
  est.y.assign(L, nullptr);
  est.z.assign(L, nullptr);
  est.w.assign(L, nullptr);
  est.u.assign(L, nullptr);
  est.v.assign(L, nullptr);
  for (int l = 0; l < L; l++) {
    size_t nb = (size_t)n(l) * cap(l);
    est.x[l] = a.take_n<double2>(nb);
    est.y[l] = a.take_n<double2>(nb);
    est.z[l] = a.take_n<double2>(nb);
    est.w[l] = a.take_n<double2>(nb);
    est.u[l] = a.take_n<double2>(nb);
    est.v[l] = a.take_n<double2>(nb);
  }
  est.qf = a.take_n<double2>(nmax);
  est.qf2 = a.take_n<double2>(nmax);
  if (desc.with_corr) {
    int nterm = 4 * L - 3;
    est.term.assign(nterm, nullptr);
    for (int i = 0; i < nterm; i++) est.term[i] = a.take_n<double2>((size_t)n(0) * nfine);
    est.eta = a.take_n<double2>((size_t)n(0) * nfine);
    const int T_ = g[0].dims[3];
    size_t np = (size_t)kSliceChunksHost * kMaxPairs * nfine * T_;
    size_t nl = (size_t)kSliceChunksHost * kMaxLoopVecs * 6 * nfine * T_;
    est.slice_partial = a.take_n<double2>(std::max(np, nl));
    est.slice_out = a.take_n<double2>((size_t)std::max(kMaxPairs, kMaxLoopVecs * 6) * nfine * T_);
  }
  // union region: solver workspaces or setup buffers
  const size_t base = a.off;
  ws64.assign(L, LevelWS{});
  ws32.assign(L, LevelWS{});
  ws16.assign(L, LevelWS{});
  for (int l = 0; l < L; l++) {
    carve_ws(a, ws64[l], MGM_PREC_F64, n(l), cap(l), m, full64);
    if (mixed) carve_ws(a, ws32[l], MGM_PREC_F32, n(l), cap(l), m, true);
  }
  if (mixed) carve_smooth16(a, ws16[0], n(0), cap(0));
  const size_t solver_end = a.off;
  a.off = base;
  tv.assign(L > 0 ? L - 1 : 0, nullptr);
  for (int l = 0; l + 1 < L; l++) tv[l] = a.take_n<double2>((size_t)n(l) * desc.ntv[l]);
  // the rough smoothing runs on chunks of kSetupChunk test vectors: its four
  // temporaries hold that many columns, not N_tv (a quarter of the memory
  // at N_tv 24 on the fine level, where four full-width copies would not fit
  // next to the hierarchy on the largest lattices)
  size_t tmp_max = 0;
  for (int l = 0; l + 1 < L; l++) tmp_max = std::max(tmp_max, (size_t)n(l) * std::min(desc.ntv[l], kSetupChunk));
  setup_v = a.take_n<double2>(tmp_max);
  setup_y = a.take_n<double2>(tmp_max);
  setup_rho = a.take_n<double2>(tmp_max);
  setup_q = a.take_n<double2>(tmp_max);
  setup_n2 = a.take_n<double>(std::max(ntv_max, 1));
  setup_qr = a.take_n<double2>(std::max(ntv_max, 1));
  setup_qq = a.take_n<double>(std::max(ntv_max, 1));
  a.off = std::max(a.off, solver_end);
}

void Hier::build() {
  for (int l = 0; l + 1 < L; l++) build_level(l, nullptr);
  ctx->sync();
}

// Transfer l and the coarse operator D_{l+1}: from the rough test-vector
// recipe, or (tvsrc != nullptr) from the given block of ntv[l] vectors of
// level l (dof-major, ntv[l] columns).
void Hier::build_level(int l, const double2* tvsrc) {
  const double2* src = tvsrc;
  if (src == nullptr) {
    rough_tv(l);
    src = tv[l];
  }
  finish_level(l, src);
}

// The rough test vectors of level l into tv[l], kSetupChunk columns at a
// time (every column is smoothed on its own, so the chunking changes nothing
// but the batch width of the launches).
void Hier::rough_tv(int l) {
  Context* c = ctx;
  const int ntv = desc.ntv[l];
  for (int k0 = 0; k0 < ntv; k0 += kSetupChunk) {
    const int nb = std::min(kSetupChunk, ntv - k0);
    Vec v = vec(l, MGM_PREC_F64, setup_v, nb);
    Vec y = v.with(setup_y), rho = v.with(setup_rho), q = v.with(setup_q);
    // Z4 starts (kind 7, probes k0 ..), then setup_steps rounds of MR_k
    // smoothing and normalisation: v <- MR(D_l, v) / |MR(D_l, v)|
    draw_z4(c, desc.seed, (uint32_t)(256 * l + 7), (uint64_t)k0, nb, g[l].V, g[l].dof, MGM_PREC_F64, setup_v);
    for (int it = 0; it < desc.setup_steps; it++) {
      b_zero(c, y);
      b_copy(c, rho, v);
      for (int k = 0; k < desc.setup_mr; k++) {
        apply(l, MGM_PREC_F64, rho.p, q.p, nb);
        b_dot_norm(c, scratch, q, rho, setup_qr, setup_qq);
        b_mr_update(c, setup_qr, setup_qq, rho, q, y);
      }
      b_norm2(c, scratch, y, setup_n2);
      b_copy(c, v, y);
      b_normalize(c, v, setup_n2, nullptr);
    }
    blk_scatter(c, setup_v, ntv, k0, nb, n(l), tv[l]);
  }
}

// P_l from a block of test vectors (block MGS2), the Galerkin D_{l+1} and
// the precision copies.
void Hier::finish_level(int l, const double2* src) {
  Context* c = ctx;
  MGM_HIP(hipMemsetAsync(d_flag, 0, sizeof(int), c->stream));
  mg_block_mgs2(c, T[l].t, src, T[l].P64, d_flag);
  int flag = 0;
  MGM_HIP(hipMemcpyAsync(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  c->sync();
  MGM_CHECK(flag == 0, MGM_ERR_RANK_DEFICIENT,
            "test vectors of level " + std::to_string(l) + " are rank deficient on some aggregate");
  if (l == 0)
    mg_galerkin_fine(c, *fine, T[0], A[1]);
  else
    mg_galerkin_coarse(c, A[l], T[l], A[l + 1]);
  mg_mfma64_pack(c, A[l + 1]);
  if (desc.mixed) {
    mg_convert_P(c, T[l]);
    mg_convert_A(c, A[l + 1]);
    mg_mfma_pack(c, A[l + 1]);
  }
  // captured coarse-grid corrections hold the old operators' launch
  // arguments only through buffer addresses, which do not move; nothing to
  // invalidate
}

}  // namespace mgm
