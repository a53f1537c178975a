// Higher-accuracy test vectors for the fine transfer (Sec. 5: test vectors
// computed to smaller eigen-residuals, 1e-1 -> 1e-4, strengthen the coarse
// space).  Reading: inverse block power on the Hermitian Q = Gamma5 D with
// the hierarchy's own solver, a Rayleigh-Ritz step after every QR, until every
// Ritz pair has rho_i = |Q v_i - theta_i v_i| / |theta_i| <= eig_tol (or a
// step limit); the Ritz vectors (ordered by |theta| ascending, phase fixed so
// that the sum of the entries is real and positive) then replace the rough
// test vectors of transfer 0, and every coarser level is rebuilt from the new
// Galerkin operator with the rough recipe.
//
// Rayleigh-Ritz without extra passes over the vectors: with Y = D V and
// Z = Gamma5 V, H = V^H Q V = Z^H Y and G = (QV)^H (QV) = Y^H Y (Gamma5 is
// unitary); for H = S diag(theta) S^H the Ritz vector V s_i has
// |Q V s_i - theta_i V s_i|^2 = s_i^H G s_i - theta_i^2.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <numeric>

#include "block.h"
#include "lib.h"

namespace mgm {

namespace {

using cd = std::complex<double>;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

__global__ void k_fill_one(double2* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(1.0, 0.0);
}

// Cyclic Jacobi for a Hermitian k x k matrix (row-major, overwritten by its
// diagonal form); S receives the eigenvectors (columns).
void jacobi_hermitian(std::vector<cd>& H, int k, std::vector<cd>& S) {
  S.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; i++) S[(size_t)i * k + i] = 1.0;
  auto at = [&](int r, int c) -> cd& { return H[(size_t)r * k + c]; };
  double fro = 0;
  for (const cd& v : H) fro += std::norm(v);
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0;
    for (int p = 0; p < k; p++)
      for (int q = p + 1; q < k; q++) off += std::norm(at(p, q));
    if (off <= 1e-30 * fro) break;
    for (int p = 0; p < k; p++)
      for (int q = p + 1; q < k; q++) {
        const cd h = at(p, q);
        const double g = std::abs(h);
        if (g == 0.0) continue;
        const cd ph = h / g;  // e^{i phi}
        const double a = at(p, p).real(), b = at(q, q).real();
        const double tau = (b - a) / (2.0 * g);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        // J = diag(1, e^{-i phi}) [[c, s], [-s, c]]
        const cd Jpp = c, Jpq = s, Jqp = -s * std::conj(ph), Jqq = c * std::conj(ph);
        for (int r = 0; r < k; r++) {  // H <- H J
          const cd hp = at(r, p), hq = at(r, q);
          at(r, p) = hp * Jpp + hq * Jqp;
          at(r, q) = hp * Jpq + hq * Jqq;
        }
        for (int r = 0; r < k; r++) {  // H <- J^H H
          const cd hp = at(p, r), hq = at(q, r);
          at(p, r) = std::conj(Jpp) * hp + std::conj(Jqp) * hq;
          at(q, r) = std::conj(Jpq) * hp + std::conj(Jqq) * hq;
        }
        for (int r = 0; r < k; r++) {  // S <- S J
          const cd sp = S[(size_t)r * k + p], sq = S[(size_t)r * k + q];
          S[(size_t)r * k + p] = sp * Jpp + sq * Jqp;
          S[(size_t)r * k + q] = sp * Jpq + sq * Jqq;
        }
        at(p, q) = 0.0;
        at(q, p) = 0.0;
      }
  }
}

}  // namespace

struct RefineWS {
  double2 *V = nullptr, *Y = nullptr, *Z = nullptr, *ones = nullptr;
  double2 *part = nullptr, *C = nullptr, *C2 = nullptr, *C3 = nullptr, *M = nullptr;
  size_t part_cap = 0;
  void layout(Arena& a, int64_t n, int k) {
    V = a.take_n<double2>((size_t)n * k);
    Y = a.take_n<double2>((size_t)n * k);
    Z = a.take_n<double2>((size_t)n * k);
    ones = a.take_n<double2>((size_t)n);
    part_cap = blk_part_entries(k, k);
    part = a.take_n<double2>(part_cap);
    C = a.take_n<double2>((size_t)k * k);
    C2 = a.take_n<double2>((size_t)k * k);
    C3 = a.take_n<double2>((size_t)k);
    M = a.take_n<double2>((size_t)k * k);
  }
};

size_t refine_workspace_bytes(const Hier& H) {
  Arena a;
  RefineWS w;
  w.layout(a, H.n(0), H.desc.ntv[0]);
  return a.off;
}

// Rayleigh-Ritz on span(V): V <- V S diag(phase); returns rho and theta.
static void rayleigh_ritz(Hier& H, RefineWS& w, int k, std::vector<double>& rho, std::vector<double>& theta) {
  Context* c = H.ctx;
  const int64_t rows = H.n(0);
  H.apply(0, MGM_PREC_F64, w.V, w.Y, k);                               // Y = D V
  blk_gather(c, w.V, k, 0, k, H.g[0].V, H.g[0].dof, true, w.Z);        // Z = Gamma5 V
  blk_ahb(c, w.Z, k, w.Y, k, rows, w.part, w.part_cap, w.C);           // H = Z^H Y
  blk_ahb(c, w.Y, k, w.Y, k, rows, w.part, w.part_cap, w.C2);          // G = Y^H Y
  blk_ahb(c, w.ones, 1, w.V, k, rows, w.part, w.part_cap, w.C3);       // u = 1^H V (column sums)
  std::vector<cd> Hm = blk_fetch(c, w.C, (size_t)k * k), G = blk_fetch(c, w.C2, (size_t)k * k),
                  u = blk_fetch(c, w.C3, (size_t)k);
  for (int i = 0; i < k; i++)
    for (int j = 0; j < k; j++) {
      const cd a = 0.5 * (Hm[(size_t)i * k + j] + std::conj(Hm[(size_t)j * k + i]));
      Hm[(size_t)i * k + j] = a;
    }
  std::vector<cd> S;
  jacobi_hermitian(Hm, k, S);
  std::vector<int> ord(k);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    return std::abs(Hm[(size_t)a * k + a].real()) < std::abs(Hm[(size_t)b * k + b].real());
  });
  rho.assign(k, 0.0);
  theta.assign(k, 0.0);
  std::vector<double2> hM((size_t)k * k);
  for (int jn = 0; jn < k; jn++) {
    const int j = ord[jn];
    const double th = Hm[(size_t)j * k + j].real();
    // s^H G s
    cd sgs = 0.0;
    for (int a = 0; a < k; a++) {
      cd gs = 0.0;
      for (int b = 0; b < k; b++) gs += G[(size_t)a * k + b] * S[(size_t)b * k + j];
      sgs += std::conj(S[(size_t)a * k + j]) * gs;
    }
    theta[jn] = th;
    rho[jn] = std::sqrt(std::max(0.0, sgs.real() - th * th)) / std::abs(th);
    // phase: the column sum of V s is u s; make it real and positive
    cd us = 0.0;
    for (int a = 0; a < k; a++) us += u[a] * S[(size_t)a * k + j];
    const cd ph = std::abs(us) > 0 ? std::conj(us) / std::abs(us) : cd(1.0);
    for (int a = 0; a < k; a++) {
      const cd m = S[(size_t)a * k + j] * ph;
      hM[(size_t)a * k + jn] = make_double2(m.real(), m.imag());
    }
  }
  MGM_HIP(hipMemcpyAsync(w.M, hM.data(), sizeof(double2) * hM.size(), hipMemcpyHostToDevice, c->stream));
  blk_rowmul(c, w.V, k, rows, w.M);
  c->sync();  // hM leaves scope
}

void refine_hierarchy(Hier& H, const mgm_refine_desc& d, const SolveCfg& power, void* ws, size_t ws_bytes,
                      mgm_refine_stats* st, double* rho_out, double* theta_out) {
  Context* c = H.ctx;
  const double t0 = now_s();
  const int k = H.desc.ntv[0];
  const int64_t rows = H.n(0);
  Arena a;
  a.base = (char*)ws;
  a.cap = ws_bytes;
  RefineWS w;
  w.layout(a, rows, k);
  hipLaunchKernelGGL(k_fill_one, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, c->stream, w.ones, rows);
  MGM_LAUNCH_CHECK();
  // the rough vectors of the hierarchy's recipe, orthonormalised
  H.rough_tv(0);
  b_copy(c, H.vec(0, MGM_PREC_F64, w.V, k), H.vec(0, MGM_PREC_F64, H.tv[0], k));
  blk_cholqr(c, w.V, k, rows, w.part, w.part_cap, w.C, w.M);
  blk_cholqr(c, w.V, k, rows, w.part, w.part_cap, w.C, w.M);
  std::vector<double> rho, theta;
  SolveOut so;
  int steps = 0;
  double rho0 = -1;
  EstWS& E = H.est;
  const int B = std::min(d.batch, H.cap(0));
  while (true) {
    rayleigh_ritz(H, w, k, rho, theta);
    const double mx = *std::max_element(rho.begin(), rho.end());
    if (rho0 < 0) rho0 = mx;
    if (mx <= d.eig_tol || steps >= d.max_iters) break;
    // power step V <- QR(D^-1 Gamma5 V), each column's solution overwriting it
    for (int c0 = 0; c0 < k; c0 += B) {
      const int nb = std::min(B, k - c0);
      blk_gather(c, w.V, k, c0, nb, H.g[0].V, H.g[0].dof, true, E.x[0]);
      solve(H, 0, power, E.x[0], E.z[0], nb, &so);
      blk_scatter(c, E.z[0], k, c0, nb, rows, w.V);
    }
    blk_cholqr(c, w.V, k, rows, w.part, w.part_cap, w.C, w.M);
    blk_cholqr(c, w.V, k, rows, w.part, w.part_cap, w.C, w.M);
    steps++;
  }
  H.finish_level(0, w.V);
  for (int l = 1; l + 1 < H.L; l++) H.build_level(l, nullptr);
  c->sync();
  if (st) {
    st->steps = steps;
    st->max_rho_start = rho0;
    st->max_rho = *std::max_element(rho.begin(), rho.end());
    st->seconds = now_s() - t0;
    st->converged = so.converged ? 1 : 0;
  }
  if (rho_out) std::copy(rho.begin(), rho.end(), rho_out);
  if (theta_out) std::copy(theta.begin(), theta.end(), theta_out);
}

}  // namespace mgm
