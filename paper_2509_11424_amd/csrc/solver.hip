// Level solves D_l x = b (the paper solves every level system to a relative
// residual of 1e-12 with a multigrid solver, Sec. 4).
//
// * FGMRES(m): Arnoldi with classical Gram-Schmidt plus one
//   re-orthogonalisation pass (a single pass in the FP32 inner solves of the
//   mixed form when their tolerance is 1e-4 or looser: the orthogonality they
//   lose stays far below that tolerance), Givens rotations and the small triangular
//   solve on the GPU; the host only reads the per-rhs residual estimate of the
//   previous step (so the GPU always has the next step queued) and the true
//   residual once per restart.
// * Preconditioner: one MG V-cycle -- minimal-residual pre-smoothing,
//   restriction P^H, a fixed number of (F)GMRES steps on the coarse level
//   (recursively preconditioned), prolongation, post-smoothing.
// * Mixed precision: FP64 defect correction r = b - D x around an FP32
//   FGMRES whose V-cycle runs on FP32 vectors (optionally FP16 fine-level
//   smoothing and BF16-MFMA coarse stencils); each inner solve is one
//   Arnoldi cycle stopped by its residual estimate, which the next FP64
//   residual checks.
#include <utility>
#include "lib.h"
#include "net.h"

namespace mgm {

// Level operator as used inside a preconditioner: FP32 coarse levels may use
// BF16 MFMA operands; the Arnoldi operator of a solve is always exact in p.
static void op_apply(Hier& H, int l, mgm_prec p, bool inner, const SolveCfg& cfg, const void* x, void* y,
                     int nrhs) {
  if (inner && l >= 1 && p == MGM_PREC_F32 && cfg.coarse_bf16 && H.A[l].Abf != nullptr)
    H.A[l].apply(MGM_PREC_BF16, x, y, nrhs);
  else
    H.apply(l, p, x, y, nrhs);
}

// FP16 fine-level smoother, fused form: the first step is the exact MR step
// (dslash with dots, then the update); every later step is one fused kernel
// that applies D, moves r and x by the previous step's MR length and forms
// the dots that give the next length (FineOp::apply_step).  r ping-pongs
// between b (the caller's scratch input, overwritten) and w.rho; the return
// value is the buffer that holds the final residual b - D y.  g: the column
// group b and y hold (b.nrhs right-hand sides from rhs g * b.nrhs on), whose
// q, rho and per-rhs dots sit at the same offsets of the workspace.
static void* mr_smooth_fused(Hier& H, Vec b, Vec y, int nu, int g = 0) {
  LevelWS& w = H.ws16[0];
  Context* c = H.ctx;
  const int64_t ge = H.n(0) * b.nrhs;  // entries of one group
  const int r0 = g * b.nrhs;
  __half2* q = (__half2*)w.q + g * ge;
  double2 *qr = w.qr + r0, *qr2 = w.qr2 + r0;
  double *qq = w.qq + r0, *qq2 = w.qq2 + r0;
  int64_t nb = H.fine->apply_dot(MGM_PREC_F16, b.p, q, b.nrhs, H.dpart);
  b_finalize_dot_norm(c, H.scratch, H.dpart, nb, b.nrhs, qr, qq);
  b_mr_update(c, qr, qq, b, b.with(q), y, nullptr, true);  // y = alpha b
  void* r = b.p;
  void* r_next = (__half2*)w.rho + g * ge;
  for (int i = 1; i < nu; i++) {
    double2* qr_prev = (i & 1) ? qr : qr2;
    double* qq_prev = (i & 1) ? qq : qq2;
    nb = H.fine->apply_step(MGM_PREC_F16, r, r_next, y.p, qr_prev, qq_prev, b.nrhs, H.dpart);
    if (i + 1 < nu)
      b_finalize_dot_norm(c, H.scratch, H.dpart, nb, b.nrhs, (i & 1) ? qr2 : qr, (i & 1) ? qq2 : qq);
    std::swap(r, r_next);
  }
  return r;
}

// MR smoothing y = S b from y = 0 (add: y += S b); the residual b - D S b
// is carried in rho, which is `res` when the caller wants it.
static void mr_smooth(Hier& H, int l, mgm_prec p, Vec b, Vec y, int nu, const SolveCfg& cfg, Vec* res = nullptr,
                      bool add = false) {
  LevelWS& w = H.ws(l, p);
  Context* c = H.ctx;
  Vec rho = res ? *res : b.with(w.rho), q = b.with(w.q);
  // the first step reads b in place of rho = b, and sets y unless adding
  if (nu <= 0) {
    if (!add) b_zero(c, y);
    b_copy(c, rho, b);
  }
  for (int i = 0; i < nu; i++) {
    const Vec cur = i == 0 ? b : rho;
    if (l == 0) {
      // fine level: q^H rho and |q|^2 come out of the dslash itself
      const int64_t nb = H.fine->apply_dot(p, cur.p, q.p, b.nrhs, H.dpart);
      b_finalize_dot_norm(c, H.scratch, H.dpart, nb, b.nrhs, w.qr, w.qq);
    } else {
      op_apply(H, l, p, true, cfg, cur.p, q.p, b.nrhs);
      b_dot_norm(c, H.scratch, q, cur, w.qr, w.qq);
    }
    b_mr_update(c, w.qr, w.qq, rho, q, y, i == 0 ? &b : nullptr, i == 0 && !add);
  }
}

static void fgmres_fixed(Hier& H, int l, mgm_prec p, Vec b, Vec x, int k, bool precond, const SolveCfg& cfg);

// the fine-level smoother of the mixed V-cycle runs in FP16 storage
static bool smooth_f16(Hier& H, int l, mgm_prec p, const SolveCfg& cfg) {
  return l == 0 && p == MGM_PREC_F32 && cfg.smooth_f16 && cfg.smooth > 0 && H.ws16.size() > 0 &&
         H.ws16[0].rho != nullptr;
}

// Column groups of the FP16 smoother: with more than 8 rhs and the fused
// step, its vectors are stored group-major ([nrhs / gs][dof][site][gs], gs
// = 8 when 8 divides nrhs, else 4 when 4 does) and smoothed one group at a
// time, so that a block of the step kernel holds all rhs of a site's run and
// reads whole 128-byte lines (8 FP16 rhs of a dof are 32 bytes; with 16 rhs
// stored together each block read half of every line, and 20 rhs have no
// marching shape with more than 4 rhs per block).  Returns the group size
// (nrhs: no groups).
static bool smooth_fusable(Hier& H, int nrhs, const SolveCfg& cfg) {
  return cfg.smooth >= 2 && H.ws16[0].qr2 != nullptr && H.fine->step_fusable(MGM_PREC_F16, nrhs);
}
static int smooth_group(Hier& H, int nrhs, const SolveCfg& cfg) {
  if (nrhs <= 8) return nrhs;
  for (int gs : {8, 4})
    if (nrhs % gs == 0 && smooth_fusable(H, gs, cfg)) return gs;
  return nrhs;
}

// Smoothing e = S r on level l.  On the fine level of the mixed V-cycle the
// smoother runs in FP16 storage: the input is scaled per rhs to unit RMS
// entries (MR is homogeneous of degree one, and FP16 keeps its full
// precision away from the subnormal range), smoothed with FP16 vectors and
// FP32 arithmetic, and scaled back into FP32.  Options:
//   res   write the residual r - D e that the smoother carries to *res (in
//         the precision of r)
//   unit  every column of r has norm 1 or 0 (a normalised Arnoldi vector):
//         no norm pass
//   add   e += S r instead of e = S r
//   sub   (FP16 smoother only) the input is r - *sub, scaled by the norms of r
//   o16   (FP16 smoother only) e and the residual stay in FP16: o16 receives
//         the FP16 correction, the FP16 residual and the per-rhs factors that
//         scale both back (e and *res are not written)
struct Smooth16 {
  const __half2* y = nullptr;
  const __half2* r = nullptr;
  const double* inv = nullptr;
  int gs = 0;  // column group size of y and r
};
static void smooth(Hier& H, int l, mgm_prec p, Vec r, Vec e, const SolveCfg& cfg, Vec* res = nullptr,
                   bool unit = false, bool add = false, const Vec* sub = nullptr, Smooth16* o16 = nullptr) {
  MGM_CHECK((sub == nullptr && o16 == nullptr) || smooth_f16(H, l, p, cfg), MGM_ERR_INVALID_ARG,
            "FP16 smoother options without the FP16 smoother");
  if (smooth_f16(H, l, p, cfg)) {
    LevelWS& w = H.ws16[0];
    Context* c = H.ctx;
    const int gs = smooth_group(H, r.nrhs, cfg);
    Vec r16 = r.as(MGM_PREC_F16, w.r), y16 = r.as(MGM_PREC_F16, w.t);
    r16.group = y16.group = gs < r.nrhs ? gs : 0;
    if (!unit) b_norm2(c, H.scratch, r, w.n2a);
    b_unit_scales(c, unit ? nullptr : w.n2a, (double)r.nsite * r.dof, r.nrhs, w.mask, w.n2b);
    if (sub)
      b_sub_scaled(c, r16, r, *sub, w.mask);
    else
      b_copy_scaled(c, r16, r, w.mask);
    void* rf = w.rho;
    if (smooth_fusable(H, gs, cfg)) {
      // each group is a plain (dof, site, gs) block
      const int64_t ge = H.n(0) * gs;
      for (int g = 0; g < r.nrhs / gs; g++) {
        Vec rg = r16, yg = y16;
        rg.group = yg.group = 0;
        rg.nrhs = yg.nrhs = gs;
        rg.p = (__half2*)w.r + g * ge;
        yg.p = (__half2*)w.t + g * ge;
        rf = mr_smooth_fused(H, rg, yg, cfg.smooth, g) == rg.p ? w.r : w.rho;
      }
    } else {
      mr_smooth(H, 0, MGM_PREC_F16, r16, y16, cfg.smooth, cfg);
    }
    if (o16) {
      o16->y = (const __half2*)y16.p;
      o16->r = (const __half2*)rf;
      o16->inv = w.n2b;
      o16->gs = gs;
      return;
    }
    if (add)
      b_add_scaled(c, e, y16, w.n2b);
    else
      b_copy_scaled(c, e, y16, w.n2b);
    if (res) b_copy_scaled(c, *res, r16.with(rf), w.n2b);
    return;
  }
  const int nu = (l > 0 && cfg.smooth_coarse > 0) ? cfg.smooth_coarse : cfg.smooth;
  mr_smooth(H, l, p, r, e, nu, cfg, res, add);
}

// e_c = (cfg.coarse_iters FGMRES steps on level lc) r_c, between the level's
// fixed coarse buffers.  Its launch sequence depends only on the level, the
// precision, the batch and the settings, so with cfg.graphs it is captured
// into a HIP graph on its second use and replayed from then on (the first,
// eager use also lets the autotuner settle every launch shape inside).
static void coarse_correction(Hier& H, int lc, mgm_prec p, Vec rc, Vec ec, const SolveCfg& cfg) {
  Context* c = H.ctx;
  const bool precond = lc < H.L - 1;
  if (!cfg.graphs || c->capturing || c->stream == nullptr) {
    fgmres_fixed(H, lc, p, rc, ec, cfg.coarse_iters, precond, cfg);
    return;
  }
  const std::string key = std::to_string(lc) + "/" + std::to_string((int)p) + "/" + std::to_string(rc.nrhs) + "/" +
                          std::to_string(cfg.coarse_iters) + "/" + std::to_string(cfg.smooth) + "/" +
                          std::to_string(cfg.smooth_coarse) + "/" +
                          std::to_string((int)cfg.coarse_bf16) + "/" + (rc.p == H.ws(lc, p).bc ? "bc" : "other");
  Hier::GraphEntry& g = H.graphs[key];
  if (g.exec) {
    MGM_HIP(hipGraphLaunch(g.exec, c->stream));
    return;
  }
  if (g.uses++ == 0 || rc.p != H.ws(lc, p).bc || ec.p != H.ws(lc, p).xc) {
    fgmres_fixed(H, lc, p, rc, ec, cfg.coarse_iters, precond, cfg);
    return;
  }
  hipGraph_t graph = nullptr;
  MGM_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  try {
    fgmres_fixed(H, lc, p, rc, ec, cfg.coarse_iters, precond, cfg);
  } catch (...) {
    c->capturing = false;
    (void)hipStreamEndCapture(c->stream, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  c->capturing = false;
  MGM_HIP(hipStreamEndCapture(c->stream, &graph));
  hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  MGM_CHECK(e == hipSuccess, MGM_ERR_HIP, std::string("graph instantiation failed: ") + hipGetErrorString(e));
  MGM_HIP(hipGraphLaunch(g.exec, c->stream));
}

void vcycle(Hier& H, int l, mgm_prec p, Vec r, Vec e, const SolveCfg& cfg, bool unit) {
  Context* c = H.ctx;
  if (l == H.L - 1) {
    fgmres_fixed(H, l, p, r, e, cfg.coarse_iters, false, cfg);
    return;
  }
  LevelWS& w = H.ws(l, p);
  const int nrhs = r.nrhs;
  Vec t = r.with(w.t);
  if (l == 0 && cfg.net != nullptr && cfg.kind == MGM_SOLVE_NET) {
    // learned smoother after the coarse-grid correction:
    // M r = e_c + N(r - D e_c), e_c = P D_c^-1 P^H r
    LevelWS& wc = H.ws(1, p);
    Vec rc = H.vec(1, p, wc.bc, nrhs), ec = H.vec(1, p, wc.xc, nrhs);
    H.T[0].restrict_(p, r.p, rc.p, nrhs);
    coarse_correction(H, 1, p, rc, ec, cfg);
    H.T[0].prolong(p, ec.p, nullptr, e.p, nrhs, 0);  // e = P e_c
    op_apply(H, 0, p, true, cfg, e.p, t.p, nrhs);
    b_xpay(c, r, nullptr, -1.0, t);
    Vec y = r.with(w.y);
    net_apply(H, *cfg.net, t, y);
    b_axpy(c, nullptr, 1.0, y, e);
    return;
  }
  // pre-smoothing; the smoother's own recursion leaves t = r - D e.  With
  // the FP16 smoother, e and t stay in FP16 and the transfers read them
  // scaled: rc = P^H t, e = e + P e_c
  Smooth16 o16;
  smooth(H, l, p, r, e, cfg, &t, unit, false, nullptr, smooth_f16(H, l, p, cfg) ? &o16 : nullptr);
  LevelWS& wc = H.ws(l + 1, p);
  Vec rc = H.vec(l + 1, p, wc.bc, nrhs), ec = H.vec(l + 1, p, wc.xc, nrhs);
  if (o16.y)
    H.T[l].restrict16(o16.r, o16.inv, (float2*)rc.p, nrhs, o16.gs);
  else
    H.T[l].restrict_(p, t.p, rc.p, nrhs);
  coarse_correction(H, l + 1, p, rc, ec, cfg);
  if (o16.y)
    H.T[l].prolong16((const float2*)ec.p, o16.y, o16.inv, (float2*)e.p, nrhs, o16.gs);
  else
    H.T[l].prolong(p, ec.p, nullptr, e.p, nrhs, 2);  // e += P e_c
  op_apply(H, l, p, true, cfg, e.p, t.p, nrhs);
  if (unit && smooth_f16(H, l, p, cfg)) {
    // e += S (r - D e): the FP16 smoother's input formed in its conversion,
    // scaled by the (unit) norms of r, as MR is homogeneous of degree one
    smooth(H, l, p, r, e, cfg, nullptr, true, true, &t);
  } else {
    b_xpay(c, r, nullptr, -1.0, t);
    smooth(H, l, p, t, e, cfg, nullptr, false, true);  // e += S t
  }
}

// Arnoldi steps from a normalised V_0 and started Givens state.  stop (host,
// per rhs) enables the lagged early exit when every estimate falls below it.
static int arnoldi(Hier& H, int l, mgm_prec p, int nrhs, int kmax, bool precond, const SolveCfg& cfg,
                   const double* stop, bool inner, bool reorth = true) {
  Context* c = H.ctx;
  LevelWS& w = H.ws(l, p);
  Givens& G = w.G;
  const int64_t stride = H.n(l) * nrhs;
  const size_t eb = prec_bytes(p);
  Vec base = H.vec(l, p, w.V, nrhs);
  double* pin = H.pinned;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (stop) {
    ev[0] = c->take_event();
    ev[1] = c->take_event();
  }
  int k = 0;
  for (int j = 0; j < kmax; j++) {
    char* Vj = (char*)w.V + (size_t)j * stride * eb;
    char* Zj = precond ? (char*)w.Z + (size_t)j * stride * eb : Vj;
    char* W = (char*)w.V + (size_t)(j + 1) * stride * eb;
    if (precond) vcycle(H, l, p, base.with(Vj), base.with(Zj), cfg, true);
    op_apply(H, l, p, inner, cfg, Zj, W, nrhs);
    Vec Wv = base.with(W);
    // classical Gram-Schmidt with one re-orthogonalisation: the first
    // subtraction and the second projection share one sweep over the basis.
    // Without reorth one pass: the Arnoldi relation still holds exactly, and
    // the orthogonality lost (about the FP32 rounding over the cancellation
    // of one step) only matters far below a loose inner tolerance.
    b_multidot(c, H.scratch, base, stride, j + 1, Wv, G.h);
    if (!reorth) {
      b_multiaxpy(c, H.scratch, base, stride, j + 1, G.h, -1.0, Wv, w.n2a);
    } else {
      if (j + 1 <= kFusedGS) {
        b_multiaxpy_dot(c, H.scratch, base, stride, j + 1, G.h, Wv, G.h2);
      } else {
        b_multiaxpy(c, H.scratch, base, stride, j + 1, G.h, -1.0, Wv, nullptr);
        b_multidot(c, H.scratch, base, stride, j + 1, Wv, G.h2);
      }
      b_multiaxpy(c, H.scratch, base, stride, j + 1, G.h2, -1.0, Wv, w.n2a);
    }
    b_normalize(c, Wv, w.n2a, nullptr);
    k_gmres_column(c, G, j, w.n2a, nrhs, reorth);
    k = j + 1;
    if (stop) {
      MGM_HIP(hipMemcpyAsync(pin + (j & 1) * nrhs, G.est, sizeof(double) * nrhs, hipMemcpyDeviceToHost,
                             c->stream));
      MGM_HIP(hipEventRecord(ev[j & 1], c->stream));
      if (j > 0) {
        MGM_HIP(hipEventSynchronize(ev[(j - 1) & 1]));
        const double* e = pin + ((j - 1) & 1) * nrhs;
        bool all = true;
        for (int r = 0; r < nrhs; r++)
          if (!(e[r] <= stop[r])) all = false;
        if (all) break;
      }
    }
  }
  if (stop) {
    c->sync();
    c->prof.pool.push_back(ev[0]);
    c->prof.pool.push_back(ev[1]);
  }
  k_gmres_solve(c, G, k, nrhs);
  return k;
}

static void fgmres_fixed(Hier& H, int l, mgm_prec p, Vec b, Vec x, int k, bool precond, const SolveCfg& cfg) {
  Context* c = H.ctx;
  LevelWS& w = H.ws(l, p);
  const int nrhs = b.nrhs;
  Vec V0 = b.with(w.V);
  b_norm2(c, H.scratch, b, w.n2a);
  // V_0 = b / |b| in one scaled copy (zero columns stay zero)
  b_unit_scales(c, w.n2a, 1.0, nrhs, w.mask, w.n2b);
  b_copy_scaled(c, V0, b, w.mask);
  k_gmres_start(c, w.G, w.n2a, nrhs);
  int kk = arnoldi(H, l, p, nrhs, std::min(k, w.m), precond, cfg, nullptr, true);
  b_multiaxpy(c, H.scratch, b.with(precond ? w.Z : w.V), H.n(l) * nrhs, kk, w.G.y, 1.0, x, nullptr, true);
}

// Restarted FGMRES to |r_i| <= tol_rel |b_i| for every rhs.  x0 = 0.
// The residual at each restart is recomputed as b - D x in precision p.
static void fgmres_tol(Hier& H, int l, mgm_prec p, Vec b, Vec x, double tol_rel, int maxcycles, int maxsteps,
                       bool precond, const SolveCfg& cfg, SolveOut* out, bool reorth = true) {
  Context* c = H.ctx;
  LevelWS& w = H.ws(l, p);
  const int nrhs = b.nrhs;
  Vec r = b.with(w.r), V0 = b.with(w.V);
  std::vector<double> b2(nrhs), r2(nrhs), stop(nrhs), beta2(nrhs), scale(nrhs);
  double* pin = H.pinned;
  b_norm2(c, H.scratch, b, w.n2a);
  MGM_HIP(hipMemcpyAsync(pin, w.n2a, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
  c->sync();
  for (int i = 0; i < nrhs; i++) b2[i] = pin[i];
  bool xset = false;  // x is written by the first solution update (zeroed if there is none)
  int steps = 0;
  for (int cyc = 0; cyc < maxcycles && steps < maxsteps; cyc++) {
    if (cyc == 0) {
      r2 = b2;  // r = b, read from b below
    } else {
      H.apply(l, p, x.p, r.p, nrhs);
      b_rsub_norm2(c, H.scratch, b, r, w.n2a);  // r = b - D x and |r|^2
      MGM_HIP(hipMemcpyAsync(pin, w.n2a, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
      c->sync();
      for (int i = 0; i < nrhs; i++) r2[i] = pin[i];
    }
    bool all = true;
    for (int i = 0; i < nrhs; i++) {
      MGM_CHECK(std::isfinite(r2[i]), MGM_ERR_NUMERIC, "non-finite residual in FGMRES");
      bool conv = b2[i] == 0.0 || std::sqrt(r2[i]) <= tol_rel * std::sqrt(b2[i]);
      if (!conv) all = false;
      beta2[i] = conv ? 0.0 : r2[i];
      scale[i] = conv ? 0.0 : 1.0 / std::sqrt(r2[i]);
      stop[i] = 0.9 * tol_rel * std::sqrt(b2[i]);
    }
    if (all) break;
    // per-rhs start: converged right-hand sides get a zero Krylov space
    for (int i = 0; i < nrhs; i++) {
      pin[i] = beta2[i];
      pin[nrhs + i] = scale[i];
    }
    MGM_HIP(hipMemcpyAsync(w.n2b, pin, sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
    MGM_HIP(hipMemcpyAsync(w.mask, pin + nrhs, sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
    b_copy_scaled(c, V0, cyc == 0 ? b : r, w.mask);
    k_gmres_start(c, w.G, w.n2b, nrhs);
    c->sync();  // the staging buffer is reused by arnoldi
    int k = arnoldi(H, l, p, nrhs, std::min(w.m, maxsteps - steps), precond, cfg, stop.data(), false, reorth);
    b_multiaxpy(c, H.scratch, b.with(precond ? w.Z : w.V), H.n(l) * nrhs, k, w.G.y, 1.0, x, nullptr, !xset);
    xset = true;
    steps += k;
    if (out) {
      out->iterations += k;
      out->restarts += 1;
    }
  }
  if (!xset) b_zero(c, x);
}

static void true_residual(Hier& H, int l, Vec b, Vec x, SolveOut* out, double tol) {
  Context* c = H.ctx;
  LevelWS& w = H.ws64[l];
  const int nrhs = b.nrhs;
  Vec r = b.with(w.r);
  H.apply(l, MGM_PREC_F64, x.p, r.p, nrhs);
  b_xpay(c, b, nullptr, -1.0, r);
  b_norm2(c, H.scratch, r, w.n2a);
  b_norm2(c, H.scratch, b, w.n2b);
  double* pin = H.pinned;
  MGM_HIP(hipMemcpyAsync(pin, w.n2a, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
  MGM_HIP(hipMemcpyAsync(pin + nrhs, w.n2b, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
  c->sync();
  double mx = 0;
  for (int i = 0; i < nrhs; i++) {
    double rel = pin[nrhs + i] > 0 ? std::sqrt(pin[i] / pin[nrhs + i]) : 0.0;
    MGM_CHECK(std::isfinite(rel), MGM_ERR_NUMERIC, "non-finite residual");
    mx = std::max(mx, rel);
  }
  out->max_rel = std::max(out->max_rel, mx);
  if (mx > tol) out->converged = false;
}

static void solve_mixed(Hier& H, int l, const SolveCfg& cfg, Vec b, Vec x, SolveOut* out) {
  Context* c = H.ctx;
  const int nrhs = b.nrhs;
  LevelWS& w64 = H.ws64[l];
  LevelWS& w32 = H.ws32[l];
  MGM_CHECK(w32.V != nullptr, MGM_ERR_INVALID_ARG, "mixed solve needs a hierarchy built with mixed != 0");
  Vec r = b.with(w64.r);
  Vec r32 = H.vec(l, MGM_PREC_F32, w32.bc, nrhs), e32 = H.vec(l, MGM_PREC_F32, w32.xc, nrhs);
  double* pin = H.pinned;
  b_norm2(c, H.scratch, b, w64.n2b);
  MGM_HIP(hipMemcpyAsync(pin, w64.n2b, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
  c->sync();
  std::vector<double> b2(pin, pin + nrhs), mask(nrhs);
  // x = 0 and r = b are not materialised: the first cycle reads b and
  // overwrites x (zeroed at the end if no cycle ran); w64.n2a holds |r|^2
  // from the fused residual update of the previous cycle
  bool x_zero = true, r_is_b = true;
  const bool precond = l < H.L - 1;
  // the learned smoother falls back to plain MG for the rest of the solve
  // when an inner solve produces non-finite values or fails to halve the
  // residual of some right-hand side
  SolveCfg cur = cfg;
  std::vector<double> prev(nrhs, -1.0);
  auto fall_back = [&](bool restart) {
    cur.net = nullptr;
    cur.kind = MGM_SOLVE_MG_MIXED;
    out->fallbacks += 1;
    if (restart) {
      x_zero = true;
      r_is_b = true;
    }
  };
  auto residual_norms = [&]() {
    if (r_is_b) {
      for (int i = 0; i < nrhs; i++) pin[i] = b2[i];
      return;
    }
    MGM_HIP(hipMemcpyAsync(pin, w64.n2a, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
    c->sync();
  };
  int steps = 0;
  for (int outer = 0; outer < 64 && steps < cfg.maxiter; outer++) {
    residual_norms();
    if (cur.net) {
      bool bad = false, nonfinite = false;
      for (int i = 0; i < nrhs; i++) {
        if (!std::isfinite(pin[i])) nonfinite = true;
        else if (prev[i] > 0 && pin[i] > 0.25 * prev[i]) bad = true;
      }
      if (nonfinite || bad) {
        fall_back(nonfinite);
        if (nonfinite) residual_norms();
      }
    }
    bool all = true;
    for (int i = 0; i < nrhs; i++) {
      MGM_CHECK(std::isfinite(pin[i]), MGM_ERR_NUMERIC, "non-finite residual in defect correction");
      bool conv = b2[i] == 0.0 || std::sqrt(pin[i]) <= cfg.tol * std::sqrt(b2[i]);
      mask[i] = conv ? 0.0 : 1.0;
      prev[i] = conv ? -1.0 : pin[i];
      if (!conv) all = false;
    }
    if (all) break;
    MGM_HIP(hipMemcpyAsync(w64.mask, mask.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, c->stream));
    b_copy_scaled(c, r32, r_is_b ? b : r, w64.mask);  // converged right-hand sides get a zero residual
    SolveOut inner;
    try {
      // one Arnoldi cycle, stopped by its residual estimate: the true
      // residual of the next defect-correction cycle checks it, so no FP32
      // restart is spent on confirming convergence
      // (one Gram-Schmidt pass when the inner tolerance is loose: 1e-4 or more)
      fgmres_tol(H, l, MGM_PREC_F32, r32, e32, cur.inner_tol, 1, cfg.maxiter - steps, precond, cur, &inner,
                 cur.inner_tol < 1e-4);
    } catch (const Error& e) {
      if (cur.net == nullptr || e.code != MGM_ERR_NUMERIC) throw;
      fall_back(true);
      continue;
    }
    steps += inner.iterations;
    out->iterations += inner.iterations;
    out->restarts += inner.restarts;
    // x += e (zero for converged right-hand sides)
    if (x_zero)
      b_copy_scaled(c, x, e32, w64.mask);
    else
      b_add_scaled(c, x, e32, w64.mask);
    x_zero = false;
    H.apply(l, MGM_PREC_F64, x.p, r.p, nrhs);
    b_rsub_norm2(c, H.scratch, b, r, w64.n2a);  // r = b - D x in FP64, and |r|^2
    r_is_b = false;
    c->sync();  // mask staging
  }
  if (x_zero) b_zero(c, x);
}

void solve(Hier& H, int l, const SolveCfg& cfg, const double2* b, double2* x, int nrhs, SolveOut* out) {
  MGM_CHECK(l >= 0 && l < H.L, MGM_ERR_INVALID_ARG, "level out of range");
  MGM_CHECK(nrhs >= 1 && nrhs <= H.cap(l), MGM_ERR_INVALID_ARG, "nrhs exceeds the capacity of the level");
  H.tv_valid = false;
  Vec bv = H.vec(l, MGM_PREC_F64, (void*)b, nrhs), xv = H.vec(l, MGM_PREC_F64, x, nrhs);
  const int m = H.desc.restart;
  switch (cfg.kind) {
    case MGM_SOLVE_GMRES:
      MGM_CHECK(H.ws64[l].V != nullptr, MGM_ERR_INVALID_ARG, "FP64 Krylov workspace not built (mixed == 1)");
      fgmres_tol(H, l, MGM_PREC_F64, bv, xv, cfg.tol, cfg.maxiter / m + 2, cfg.maxiter, false, cfg, out);
      break;
    case MGM_SOLVE_MG:
      MGM_CHECK(H.ws64[l].V != nullptr, MGM_ERR_INVALID_ARG, "FP64 Krylov workspace not built (mixed == 1)");
      fgmres_tol(H, l, MGM_PREC_F64, bv, xv, cfg.tol, cfg.maxiter / m + 2, cfg.maxiter, l < H.L - 1, cfg, out);
      break;
    case MGM_SOLVE_MG_MIXED:
    case MGM_SOLVE_NET:
      solve_mixed(H, l, cfg, bv, xv, out);
      break;
    default:
      throw Error(MGM_ERR_INVALID_ARG, "unknown solver kind");
  }
  true_residual(H, l, bv, xv, out, cfg.tol);
}

}  // namespace mgm
