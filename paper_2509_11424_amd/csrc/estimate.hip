// Hutchinson estimators of every decomposition with per-term variances.
//
// tr(D^-1):  plain x^H D^-1 x (Sec. 1, eq. Hutchinson);
//   oblique  M_l = D_l^-1 - P_l D_{l+1}^-1 P_l^H (Sec. 2.2, eq. oblique-deflation);
//   orthogonal O_l = (I - P P^H) D_l^-1 (I - P P^H) (two-sided, Sec. 3),
//              F_l = P_l^H D_l^-1 P_l - D_{l+1}^-1, coarsest D_L^-1
//              (Sec. 3, eqs. OandF_def and the decomposition after them).
// Connected correlator (Sec. 4.1): G_rs(t) = (1/T) sum_t' tr(B_r(t+t',t) G5
//   B_s(t',t+t') G5) = (1/T) sum_t' E[(B~_s eta_t')^H_{t+t'} (B_r eta_t')_{t+t'}]
//   with B~ = G5 B^H G5 and time-diluted Z4 sources eta_t'.  Orthogonal terms
//   J_l = (I-Pi)D^-1, K_l = Pi D^-1 - P D_{l+1}^-1 P^H (J~ = D^-1 (I-Pi),
//   K~ = D^-1 Pi - P D_{l+1}^-1 P^H) share two solves per level and source:
//   u = D_l^-1 (I-Pi) y, v = D_l^-1 Pi y, w = D_{l+1}^-1 P^H y:
//   J y = (I-Pi)(u+v), J~ y = u, K y = Pi(u+v) - P w, K~ y = v - P w.
//   The accumulated transfer embedding the level-l terms is P_0 ... P_{l-1}.
// Loops (Sec. 4.3): X(t, Gamma) = sum_{x in t} eta(x)^H Gamma (B eta)(x).
// Variance (Sec. 4): sum |X - mean|^2 / (N - 1).
#include <chrono>

#include "lib.h"

namespace mgm {

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Run {
  Hier& H;
  const mgm_estimate_desc& d;
  SolveCfg cfg;
  SolveOut so;
  Context* c;
  int L;
  Run(Hier& h, const mgm_estimate_desc& dd) : H(h), d(dd), c(h.ctx), L(h.L) {
    cfg.tol = d.solve.tol;
    cfg.maxiter = d.solve.maxiter;
    cfg.kind = d.solve.kind;
    cfg.smooth = d.solve.smooth;
    cfg.smooth_coarse = d.solve.smooth_coarse;
    cfg.coarse_iters = d.solve.coarse_iters;
    cfg.inner_tol = d.solve.inner_tol > 0 ? d.solve.inner_tol : 1e-5;
    cfg.coarse_bf16 = d.solve.coarse_bf16 != 0;
    cfg.smooth_f16 = d.solve.smoother_f16 != 0;
    cfg.graphs = d.solve.graphs != 0;
    cfg.net = (Net*)d.solve.net;
  }
  Vec v(int l, void* p, int nb) { return H.vec(l, MGM_PREC_F64, p, nb); }
  // right-hand sides per launch for probe group g, bounded by level capacity
  int batch(int g, int level_cap) const {
    int b = d.batch_level[g] > 0 ? d.batch_level[g] : d.batch;
    MGM_CHECK(b >= 1 && b <= H.cap(level_cap), MGM_ERR_INVALID_ARG,
              "batch exceeds the right-hand-side capacity of level " + std::to_string(level_cap));
    return b;
  }
  void solve(int l, const double2* b, double2* x, int nb) { mgm::solve(H, l, cfg, b, x, nb, &so); }
  // probes of stream (ls, kind) on the lattice of level `lat`, from the
  // estimate's distribution; slice >= 0: one time slice (fine lattice),
  // colour >= 0: one colour of the probing pattern (fine lattice)
  void z4(int ls, int kind, int lat, uint64_t first, int nb, double2* out, int slice = -1, int colour = -1) {
    MGM_CHECK(first + (uint64_t)nb <= (1ull << 32), MGM_ERR_INVALID_ARG, "probe indices must be below 2^32");
    NoiseMask mk;
    mk.slice = slice;
    mk.sites_per_slice = (int64_t)H.g[0].dims[0] * H.g[0].dims[1] * H.g[0].dims[2];
    if (colour >= 0) {
      mk.colour = colour;
      mk.p = d.probing;
      mk.X = H.g[0].dims[0];
      mk.Y = H.g[0].dims[1];
      mk.Z = H.g[0].dims[2];
    }
    draw_noise(c, d.noise, d.seed, (uint32_t)(256 * ls + kind), first, nb, H.g[lat].V, H.g[lat].dof, MGM_PREC_F64,
               out, mk);
  }
  // out = a^H b per rhs (device), then fetched with the other values
  void dot(int l, const double2* a, const double2* b, int nb, double2* out) {
    b_dot(c, H.scratch, v(l, (void*)a, nb), v(l, (void*)b, nb), out);
  }
  std::vector<std::complex<double>> fetch(const double2* dev, int nb) {
    std::vector<double2> h(nb);
    MGM_HIP(hipMemcpyAsync(h.data(), dev, sizeof(double2) * nb, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    std::vector<std::complex<double>> o(nb);
    for (int i = 0; i < nb; i++) o[i] = {h[i].x, h[i].y};
    return o;
  }
  // y_c = P_l^H x, y = P_l x_c, y = (I - P P^H) x, y = P P^H x
  void restrict_(int l, const double2* x, double2* yc, int nb) { H.T[l].restrict_(MGM_PREC_F64, x, yc, nb); }
  void prolong(int l, const double2* xc, double2* y, int nb) {
    H.T[l].prolong(MGM_PREC_F64, xc, nullptr, y, nb, 0);
  }
  void prolong_sub(int l, const double2* xc, const double2* x, double2* y, int nb) {
    H.T[l].prolong(MGM_PREC_F64, xc, x, y, nb, 1);
  }
  // to the fine lattice: P_0 ... P_{l-1} src -> dst (uses est.x[1..l-1] as scratch)
  void to_fine(int l, const double2* src, double2* dst, int nb) {
    if (l == 0) {
      b_copy(c, v(0, dst, nb), v(0, (void*)src, nb));
      return;
    }
    const double2* cur = src;
    for (int k = l - 1; k >= 0; k--) {
      double2* out = k == 0 ? dst : H.est.x[k];
      prolong(k, cur, out, nb);
      cur = out;
    }
  }
};

struct TermAcc {
  std::vector<std::complex<double>> s;  // [probe][ngamma][T]
  double seconds = 0;
  int64_t n = 0;
};

}  // namespace

// -------------------------------------------------------------- term lists

static int nterms_for(int obs, int dec, int L) {
  if (dec == MGM_DEC_PLAIN) return 1;
  if (obs == MGM_OBS_TRACE) return dec == MGM_DEC_OBLIQUE ? L : 2 * L - 1;
  return dec == MGM_DEC_OBLIQUE ? L : 2 * L - 1;
}

// finest level a term (or correlator pair) touches
static int term_level(int dec, int L, int r) {
  if (dec == MGM_DEC_PLAIN) return 0;
  if (dec == MGM_DEC_OBLIQUE) return r;
  if (r == 2 * L - 2) return L - 1;
  return r < L - 1 ? r : r - (L - 1);
}

mgm_estimate_sizes estimate_sizes(const Hier& H, const mgm_estimate_desc& d) {
  mgm_estimate_sizes s{};
  const int L = H.L;
  if (d.decomposition == MGM_DEC_DEFLATED) {
    // the stochastic term and the exact tr(V^H D^-1 V) (one value)
    s.nterms = 2;
    s.T = 1;
    s.ngamma = 1;
    s.nsamples = (int64_t)d.nprobe[0] + 1;
    return s;
  }
  int R = nterms_for(d.observable, d.decomposition, L);
  s.nterms = d.observable == MGM_OBS_CORR_PS ? R * R : R;
  s.T = d.observable == MGM_OBS_TRACE ? 1 : H.g[0].dims[3];
  s.ngamma = d.observable == MGM_OBS_LOOPS ? 6 : 1;
  int64_t tot = 0;
  for (int q = 0; q < s.nterms; q++) {
    int lv;
    if (d.observable == MGM_OBS_CORR_PS)
      lv = std::min(term_level(d.decomposition, L, q / R), term_level(d.decomposition, L, q % R));
    else
      lv = term_level(d.decomposition, L, q);
    tot += d.nprobe[lv];
  }
  s.nsamples = tot * s.ngamma * s.T;
  return s;
}

// ------------------------------------------------------------------- trace

static void trace_terms(Run& R, std::vector<TermAcc>& acc) {
  Hier& H = R.H;
  EstWS& E = H.est;
  const int L = R.L, dec = R.d.decomposition;
  const int nt = (int)acc.size();
  for (int term = 0; term < nt; term++) {
    const int lv = term_level(dec, L, term);
    const int N = R.d.nprobe[lv];
    const int B = R.batch(lv, lv);
    TermAcc& A = acc[term];
    double t0 = now_s();
    for (int b0 = 0; b0 < N; b0 += B) {
      const int nb = std::min(B, N - b0);
      const uint64_t first = R.d.first_probe + b0;
      std::vector<std::complex<double>> X;
      if (dec == MGM_DEC_PLAIN) {
        R.z4(0, 0, 0, first, nb, E.x[0]);
        R.solve(0, E.x[0], E.z[0], nb);
        R.dot(0, E.x[0], E.z[0], nb, E.qf);
        X = R.fetch(E.qf, nb);
      } else if ((dec == MGM_DEC_OBLIQUE && term == L - 1) || (dec == MGM_DEC_ORTHOGONAL && term == 2 * L - 2)) {
        R.z4(L - 1, 4, L - 1, first, nb, E.x[L - 1]);
        R.solve(L - 1, E.x[L - 1], E.z[L - 1], nb);
        R.dot(L - 1, E.x[L - 1], E.z[L - 1], nb, E.qf);
        X = R.fetch(E.qf, nb);
      } else if (dec == MGM_DEC_OBLIQUE) {  // M_l
        const int l = term;
        R.z4(l, 3, l, first, nb, E.x[l]);
        R.solve(l, E.x[l], E.z[l], nb);
        R.restrict_(l, E.x[l], E.x[l + 1], nb);
        R.solve(l + 1, E.x[l + 1], E.w[l + 1], nb);
        R.dot(l, E.x[l], E.z[l], nb, E.qf);
        R.dot(l + 1, E.x[l + 1], E.w[l + 1], nb, E.qf2);
        X = R.fetch(E.qf, nb);
        auto X2 = R.fetch(E.qf2, nb);
        for (int i = 0; i < nb; i++) X[i] -= X2[i];
      } else if (term < L - 1) {  // O_l
        const int l = term;
        R.z4(l, 1, l, first, nb, E.x[l]);
        R.restrict_(l, E.x[l], E.w[l + 1], nb);
        R.prolong_sub(l, E.w[l + 1], E.x[l], E.y[l], nb);  // y = (I - P P^H) x
        R.solve(l, E.y[l], E.z[l], nb);
        R.dot(l, E.y[l], E.z[l], nb, E.qf);
        X = R.fetch(E.qf, nb);
      } else {  // F_l
        const int l = term - (L - 1);
        R.z4(l, 2, l + 1, first, nb, E.x[l + 1]);
        R.prolong(l, E.x[l + 1], E.y[l], nb);  // P x
        R.solve(l, E.y[l], E.z[l], nb);
        R.solve(l + 1, E.x[l + 1], E.w[l + 1], nb);
        R.dot(l, E.y[l], E.z[l], nb, E.qf);
        R.dot(l + 1, E.x[l + 1], E.w[l + 1], nb, E.qf2);
        X = R.fetch(E.qf, nb);
        auto X2 = R.fetch(E.qf2, nb);
        for (int i = 0; i < nb; i++) X[i] -= X2[i];
      }
      for (auto& x : X) A.s.push_back(x);
    }
    A.seconds = now_s() - t0;
    A.n = N;
  }
}

// ------------------------------------------------------- deflated trace

// Sec. 2.1, eq. deflated-estimator: X = x^H (I - V V^H) D^-1 x
//   = x^H y - (V^H x)^H (V^H y), y = D^-1 x, plus tr(V^H D^-1 V).
static void deflated_terms(Run& R, Defl& F, std::vector<TermAcc>& acc) {
  Hier& H = R.H;
  EstWS& E = H.est;
  const int N = R.d.nprobe[0];
  const int B = R.batch(0, 0);
  const int k = F.k;
  TermAcc& A = acc[0];
  double t0 = now_s();
  for (int b0 = 0; b0 < N; b0 += B) {
    const int nb = std::min(B, N - b0);
    R.z4(0, kStreamDeflProbe, 0, R.d.first_probe + b0, nb, E.x[0]);
    R.solve(0, E.x[0], E.z[0], nb);
    R.dot(0, E.x[0], E.z[0], nb, E.qf);
    F.vh_times(E.x[0], nb, F.C);
    F.vh_times(E.z[0], nb, F.C2);
    auto X = R.fetch(E.qf, nb);
    auto a = R.fetch(F.C, k * nb);
    auto c = R.fetch(F.C2, k * nb);
    for (int j = 0; j < nb; j++) {
      std::complex<double> s = 0.0;
      for (int i = 0; i < k; i++) s += std::conj(a[(size_t)i * nb + j]) * c[(size_t)i * nb + j];
      A.s.push_back(X[j] - s);
    }
  }
  A.seconds = now_s() - t0;
  A.n = N;
  acc[1].s.push_back(F.exact);
  acc[1].seconds = F.exact_seconds;
  acc[1].n = 1;
}

// ---------------------------------------------------- fine term vectors

// Computes the fine-lattice vectors B_r eta and B~_r eta for every term r
// with term level >= g (others left untouched).  Bv[r], Bt[r]: device
// pointers to fill.  eta is the fine source.
static void term_vectors(Run& R, int g, const double2* eta, int nb, const std::vector<double2*>& Bv,
                         const std::vector<double2*>& Bt, bool need_tilde) {
  Hier& H = R.H;
  EstWS& E = H.est;
  const int L = R.L, dec = R.d.decomposition;
  // y_l = P_{l-1}^H ... P_0^H eta for l >= g (y_0 = eta)
  const double2* yl[MGM_MAX_LEVELS];
  yl[0] = eta;
  for (int l = 0; l + 1 < L && l + 1 <= L - 1; l++) {
    if (l + 1 > L - 1) break;
    R.restrict_(l, yl[l], E.y[l + 1], nb);
    yl[l + 1] = E.y[l + 1];
  }
  if (dec == MGM_DEC_PLAIN) {
    R.solve(0, eta, E.z[0], nb);
    b_copy(R.c, R.v(0, Bv[0], nb), R.v(0, E.z[0], nb));
    return;
  }
  if (dec == MGM_DEC_OBLIQUE) {
    // z_l = D_l^-1 y_l, B_l y = z_l - P_l z_{l+1}, B_{L-1} y = z_{L-1}
    for (int l = g; l < L; l++) R.solve(l, yl[l], E.z[l], nb);
    for (int l = g; l < L; l++) {
      if (l < L - 1) {
        // u_l = z_l - P z_{l+1}
        R.prolong_sub(l, E.z[l + 1], E.z[l], E.u[l], nb);
        R.to_fine(l, E.u[l], Bv[l], nb);
      } else {
        R.to_fine(l, E.z[l], Bv[l], nb);
      }
    }
    return;
  }
  // orthogonal: u_l = D^-1 (I - Pi) y, v_l = D^-1 Pi y for g <= l < L-1;
  // coarsest w = D_{L-1}^-1 y_{L-1}
  for (int l = g; l < L - 1; l++) {
    R.restrict_(l, yl[l], E.w[l + 1], nb);
    R.prolong_sub(l, E.w[l + 1], yl[l], E.x[l], nb);  // (I - Pi) y  (x used as scratch)
    R.solve(l, E.x[l], E.u[l], nb);
    R.prolong(l, E.w[l + 1], E.x[l], nb);             // Pi y
    R.solve(l, E.x[l], E.v[l], nb);
  }
  R.solve(L - 1, yl[L - 1], E.z[L - 1], nb);  // coarsest
  // w_l = D_{l+1}^-1 y_{l+1} = u_{l+1} + v_{l+1}, or the coarsest solve
  for (int l = L - 2; l >= g; l--) {
    double2* wl = E.w[l + 1];
    if (l + 1 == L - 1) {
      b_copy(R.c, R.v(L - 1, wl, nb), R.v(L - 1, E.z[L - 1], nb));
    } else {
      b_copy(R.c, R.v(l + 1, wl, nb), R.v(l + 1, E.u[l + 1], nb));
      b_axpy(R.c, nullptr, 1.0, R.v(l + 1, E.v[l + 1], nb), R.v(l + 1, wl, nb));
    }
    Vec uv = R.v(l, E.z[l], nb);  // z_l = u + v = D_l^-1 y_l
    b_copy(R.c, uv, R.v(l, E.u[l], nb));
    b_axpy(R.c, nullptr, 1.0, R.v(l, E.v[l], nb), uv);
    // J y = (I - Pi)(u + v)
    R.restrict_(l, E.z[l], E.x[l + 1], nb);
    R.prolong_sub(l, E.x[l + 1], E.z[l], E.x[l], nb);
    R.to_fine(l, E.x[l], Bv[l], nb);
    // K y = Pi(u + v) - P w = P (P^H (u+v) - w)
    b_axpy(R.c, nullptr, -1.0, R.v(l + 1, wl, nb), R.v(l + 1, E.x[l + 1], nb));
    R.prolong(l, E.x[l + 1], E.x[l], nb);
    R.to_fine(l, E.x[l], Bv[L - 1 + l], nb);
    if (need_tilde) {
      // J~ y = u ; K~ y = v - P w
      R.to_fine(l, E.u[l], Bt[l], nb);
      R.prolong_sub(l, wl, E.v[l], E.x[l], nb);
      R.to_fine(l, E.x[l], Bt[L - 1 + l], nb);
    }
  }
  R.to_fine(L - 1, E.z[L - 1], Bv[2 * L - 2], nb);
}

// ----------------------------------------------------------- correlator

static void corr_terms(Run& R, std::vector<TermAcc>& acc) {
  Hier& H = R.H;
  EstWS& E = H.est;
  const int L = R.L, dec = R.d.decomposition;
  const int Rn = nterms_for(MGM_OBS_CORR_PS, dec, L);
  const int T = H.g[0].dims[3];
  const int64_t Vs = H.g[0].V / T;
  MGM_CHECK(!E.term.empty(), MGM_ERR_INVALID_ARG, "hierarchy built without with_corr");
  std::vector<double2*> Bv(Rn), Bt(Rn);
  const bool orth = dec == MGM_DEC_ORTHOGONAL;
  for (int r = 0; r < Rn; r++) Bv[r] = E.term[r];
  for (int r = 0; r < Rn; r++) Bt[r] = Bv[r];
  if (orth)
    for (int l = 0; l < L - 1; l++) {
      Bt[l] = E.term[Rn + l];
      Bt[L - 1 + l] = E.term[Rn + (L - 1) + l];
    }
  for (int g = 0; g < L; g++) {
    if (dec == MGM_DEC_PLAIN && g > 0) break;
    std::vector<int> pairs;
    for (int r = 0; r < Rn; r++)
      for (int s = 0; s < Rn; s++)
        if (std::min(term_level(dec, L, r), term_level(dec, L, s)) == g) pairs.push_back(r * Rn + s);
    if (pairs.empty()) continue;
    const int N = R.d.nprobe[g];
    const int B = R.batch(g, 0);  // sources live on the fine lattice
    double t0 = now_s();
    for (int b0 = 0; b0 < N; b0 += B) {
      const int nb = std::min(B, N - b0);
      std::vector<std::complex<double>> X((size_t)pairs.size() * nb * T, 0.0);
      for (int tp = 0; tp < T; tp++) {
        R.z4(g, 5, 0, R.d.first_probe + b0, nb, E.eta, tp);
        term_vectors(R, g, E.eta, nb, Bv, Bt, orth);
        for (size_t p0 = 0; p0 < pairs.size(); p0 += kMaxPairs) {
          const int np = (int)std::min(pairs.size() - p0, (size_t)kMaxPairs);
          SliceArgs sa{};
          // distinct vectors referenced by this chunk
          std::vector<int> ra, sb;
          for (int i = 0; i < np; i++) {
            int r = pairs[p0 + i] / Rn, s = pairs[p0 + i] % Rn;
            auto ia = std::find(ra.begin(), ra.end(), r);
            if (ia == ra.end()) { ra.push_back(r); ia = ra.end() - 1; }
            auto ib = std::find(sb.begin(), sb.end(), s);
            if (ib == sb.end()) { sb.push_back(s); ib = sb.end() - 1; }
            sa.ri[i] = (int)(ia - ra.begin());
            sa.si[i] = (int)(ib - sb.begin());
          }
          MGM_CHECK((int)ra.size() <= kMaxSliceVecs && (int)sb.size() <= kMaxSliceVecs, MGM_ERR_INVALID_ARG,
                    "too many correlator terms");
          for (size_t i = 0; i < ra.size(); i++) sa.a[i] = Bv[ra[i]];
          for (size_t i = 0; i < sb.size(); i++) sa.b[i] = Bt[sb[i]];
          sa.npairs = np;
          slice_pairs(R.c, sa, Vs, T, nb, E.slice_partial, E.slice_out);
          std::vector<double2> h((size_t)np * nb * T);
          MGM_HIP(hipMemcpyAsync(h.data(), E.slice_out, sizeof(double2) * h.size(), hipMemcpyDeviceToHost,
                                 R.c->stream));
          R.c->sync();
          for (int i = 0; i < np; i++)
            for (int k = 0; k < nb; k++)
              for (int t = 0; t < T; t++) {
                double2 v = h[((size_t)i * nb + k) * T + (t + tp) % T];
                X[((p0 + i) * nb + k) * T + t] += std::complex<double>(v.x, v.y) / (double)T;
              }
        }
      }
      for (size_t i = 0; i < pairs.size(); i++) {
        TermAcc& A = acc[pairs[i]];
        for (int k = 0; k < nb; k++)
          for (int t = 0; t < T; t++) A.s.push_back(X[(i * nb + k) * T + t]);
      }
    }
    double dt = now_s() - t0;
    for (int q : pairs) {
      acc[q].seconds = dt / pairs.size();
      acc[q].n = N;
    }
  }
}

// ----------------------------------------------------------------- loops

static void loop_terms(Run& R, std::vector<TermAcc>& acc) {
  Hier& H = R.H;
  EstWS& E = H.est;
  const int L = R.L, dec = R.d.decomposition;
  const int Rn = nterms_for(MGM_OBS_LOOPS, dec, L);
  const int T = H.g[0].dims[3];
  const int64_t Vs = H.g[0].V / T;
  MGM_CHECK(!E.term.empty(), MGM_ERR_INVALID_ARG, "hierarchy built without with_corr");
  std::vector<double2*> Bv(Rn);
  for (int r = 0; r < Rn; r++) Bv[r] = E.term[r];
  for (int g = 0; g < L; g++) {
    if (dec == MGM_DEC_PLAIN && g > 0) break;
    std::vector<int> terms;
    for (int r = 0; r < Rn; r++)
      if (term_level(dec, L, r) == g) terms.push_back(r);
    if (terms.empty()) continue;
    const int N = R.d.nprobe[g];
    const int B = R.batch(g, 0);  // sources live on the fine lattice
    double t0 = now_s();
    // probing: one source per colour of the p^4 pattern, values summed
    const int p = R.d.probing > 1 ? R.d.probing : 1;
    const int ncol = p > 1 ? p * p * p * p : 1;
    for (int b0 = 0; b0 < N; b0 += B) {
      const int nb = std::min(B, N - b0);
      std::vector<std::complex<double>> X((size_t)terms.size() * 6 * nb * T, 0.0);
      for (int col = 0; col < ncol; col++) {
        R.z4(g, 6, 0, R.d.first_probe + b0, nb, E.eta, -1, p > 1 ? col : -1);
        term_vectors(R, g, E.eta, nb, Bv, Bv, false);
        LoopArgs la{};
        la.eta = E.eta;
        la.nvec = (int)terms.size();
        for (size_t i = 0; i < terms.size(); i++) la.psi[i] = Bv[terms[i]];
        loop_gamma(R.c, la, Vs, T, nb, E.slice_partial, E.slice_out);
        std::vector<double2> h((size_t)terms.size() * 6 * nb * T);
        MGM_HIP(hipMemcpyAsync(h.data(), E.slice_out, sizeof(double2) * h.size(), hipMemcpyDeviceToHost,
                               R.c->stream));
        R.c->sync();
        for (size_t e = 0; e < h.size(); e++) X[e] += std::complex<double>(h[e].x, h[e].y);
      }
      for (size_t i = 0; i < terms.size(); i++)
        for (int k = 0; k < nb; k++)
          for (int gm = 0; gm < 6; gm++)
            for (int t = 0; t < T; t++) acc[terms[i]].s.push_back(X[(((size_t)i * 6 + gm) * nb + k) * T + t]);
    }
    double dt = now_s() - t0;
    for (int q : terms) {
      acc[q].seconds = dt / terms.size();
      acc[q].n = N;
    }
  }
}

// -------------------------------------------------------------- driver

void estimate(Hier& H, const mgm_estimate_desc& d, mgm_estimate_result* out) {
  MGM_CHECK(d.batch >= 1, MGM_ERR_INVALID_ARG, "batch must be >= 1");
  MGM_CHECK(d.decomposition >= 0 && d.decomposition <= 3 && d.observable >= 0 && d.observable <= 2,
            MGM_ERR_INVALID_ARG, "bad observable or decomposition");
  MGM_CHECK(d.noise >= MGM_NOISE_Z4 && d.noise <= MGM_NOISE_GAUSS, MGM_ERR_INVALID_ARG, "unknown probe distribution");
  MGM_CHECK(d.probing >= 0 && d.probing <= 8, MGM_ERR_INVALID_ARG, "probing distance must be 0..8");
  if (d.probing > 1) {
    MGM_CHECK(d.observable == MGM_OBS_LOOPS, MGM_ERR_INVALID_ARG, "probing sources are for loops");
    for (int m = 0; m < 4; m++)
      MGM_CHECK(H.g[0].dims[m] % d.probing == 0, MGM_ERR_SHAPE, "probing distance must divide the fine lattice");
  }
  Defl* defl = nullptr;
  if (d.decomposition == MGM_DEC_DEFLATED) {
    MGM_CHECK(d.observable == MGM_OBS_TRACE, MGM_ERR_INVALID_ARG, "the deflated decomposition estimates the trace");
    MGM_CHECK(d.deflation != nullptr && d.deflation->f.H == &H, MGM_ERR_INVALID_ARG,
              "the deflated decomposition needs a basis built on this hierarchy");
    defl = &d.deflation->f;
  }
  for (int l = 0; l < H.L; l++) MGM_CHECK(d.nprobe[l] >= 0, MGM_ERR_INVALID_ARG, "negative probe count");
  mgm_estimate_sizes sz = estimate_sizes(H, d);
  Run R(H, d);
  std::vector<TermAcc> acc(sz.nterms);
  if (defl != nullptr)
    deflated_terms(R, *defl, acc);
  else if (d.observable == MGM_OBS_TRACE)
    trace_terms(R, acc);
  else if (d.observable == MGM_OBS_CORR_PS)
    corr_terms(R, acc);
  else
    loop_terms(R, acc);
  const int G = sz.ngamma, T = sz.T, K = G * T;
  std::vector<std::complex<double>> tot_mean(K, 0.0);
  std::vector<double> tot_var(K, 0.0);
  int64_t off = 0;
  for (int q = 0; q < sz.nterms; q++) {
    TermAcc& A = acc[q];
    const int64_t N = A.n;
    if (out->n) out->n[q] = N;
    if (out->cost_s) out->cost_s[q] = N > 0 ? A.seconds / N : 0.0;
    for (int k = 0; k < K; k++) {
      std::complex<double> mu = 0;
      for (int64_t i = 0; i < N; i++) mu += A.s[i * K + k];
      if (N > 0) mu /= (double)N;
      double var = 0;
      for (int64_t i = 0; i < N; i++) var += std::norm(A.s[i * K + k] - mu);
      var = N > 1 ? var / (double)(N - 1) : 0.0;
      if (out->mean) {
        out->mean[2 * ((int64_t)q * K + k)] = mu.real();
        out->mean[2 * ((int64_t)q * K + k) + 1] = mu.imag();
      }
      if (out->var) out->var[(int64_t)q * K + k] = var;
      tot_mean[k] += mu;
      if (N > 0) tot_var[k] += var / (double)N;
    }
    if (out->samples)
      for (int64_t i = 0; i < N * K; i++) {
        out->samples[2 * (off + i)] = A.s[i].real();
        out->samples[2 * (off + i) + 1] = A.s[i].imag();
      }
    off += N * K;
  }
  for (int k = 0; k < K; k++) {
    if (out->total_mean) {
      out->total_mean[2 * k] = tot_mean[k].real();
      out->total_mean[2 * k + 1] = tot_mean[k].imag();
    }
    if (out->total_var) out->total_var[k] = tot_var[k];
  }
  out->stats.iterations = R.so.iterations;
  out->stats.restarts = R.so.restarts;
  out->stats.fallbacks = R.so.fallbacks;
  out->stats.max_rel_residual = R.so.max_rel;
  if (!R.so.converged) throw Error(MGM_ERR_NOT_CONVERGED, "some solve missed the tolerance");
}

}  // namespace mgm
