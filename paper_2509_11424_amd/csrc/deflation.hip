// Inexact deflation of the Hutchinson estimator of tr(D^-1) (Sec. 2.1, "Deflation"
// and "Deflation for the Dirac operator", eq. deflated-estimator; setup as in
// Sec. 4.2):
//
//   tr(D^-1) = E[x^H (I - V V^H) D^-1 x] + tr(V^H D^-1 V),
//
// V (n x k, orthonormal columns) approximating the eigenvectors of the
// Hermitian Gamma5 D of smallest |eigenvalue|, from inverse block power steps
// V <- QR(D^-1 Gamma5 V) starting from k orthonormalised Z4 columns.
//
// Layout: V is one dof-major block of k vectors, element (dof, site, column)
// at (dof * V + site) * k + column, the layout of a batch of k right-hand
// sides, so the start block is one Z4 draw and a batch of columns is a
// strided gather.  Products with V (the Gram matrix V^H V, V^H x for a batch
// of probes) and the QR (CholeskyQR applied twice: the unique Q with positive
// diag(R)) are the block operations of block.hip.
#include <chrono>
#include <cmath>
#include <complex>

#include "block.h"
#include "lib.h"

namespace mgm {

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

size_t Defl::part_entries(int k, int kb_max) { return blk_part_entries(k, std::max(k, kb_max)); }

void Defl::layout(Arena& a) {
  const int64_t n = H->n(0);
  const int kbm = std::max(k, H->cap(0));
  V = a.take_n<double2>((size_t)n * k);
  part_cap = part_entries(k, H->cap(0));
  part = a.take_n<double2>(part_cap);
  C = a.take_n<double2>((size_t)k * kbm);
  C2 = a.take_n<double2>((size_t)k * kbm);
  M = a.take_n<double2>((size_t)k * k);
}

void Defl::gather(int c0, int b, bool g5, double2* out) {
  blk_gather(H->ctx, V, k, c0, b, H->g[0].V, H->g[0].dof, g5, out);
}

void Defl::scatter(int c0, int b, const double2* in) { blk_scatter(H->ctx, in, k, c0, b, H->n(0), V); }

void Defl::vh_times(const double2* X, int nb, double2* out) {
  blk_ahb(H->ctx, V, k, X, nb, H->n(0), part, part_cap, out);
}

void Defl::cholqr() { blk_cholqr(H->ctx, V, k, H->n(0), part, part_cap, C, M); }

void Defl::build(const mgm_deflation_desc& d, const SolveCfg& power, const SolveCfg& exact_cfg) {
  Hier& h = *H;
  Context* c = h.ctx;
  EstWS& E = h.est;
  const double t0 = now_s();
  const LGeom& g = h.g[0];
  // start block: k Z4 columns (kind 9, probe index = column), orthonormalised
  draw_z4(c, d.seed, (uint32_t)kStreamDeflBasis, 0, k, g.V, g.dof, MGM_PREC_F64, V);
  cholqr();
  cholqr();
  for (int it = 0; it < d.power_iters; it++) {
    // V <- D^-1 Gamma5 V, column batch by column batch (each column's input
    // is read only by its own solve, so the solution overwrites it)
    for (int c0 = 0; c0 < k; c0 += batch) {
      const int nb = std::min(batch, k - c0);
      gather(c0, nb, true, E.x[0]);
      solve(h, 0, power, E.x[0], E.z[0], nb, &so);
      scatter(c0, nb, E.z[0]);
    }
    cholqr();
    cholqr();
  }
  setup_seconds = now_s() - t0;
  // tr(V^H D^-1 V) = sum_j v_j^H D^-1 v_j
  const double t1 = now_s();
  std::complex<double> tr = 0.0;
  for (int c0 = 0; c0 < k; c0 += batch) {
    const int nb = std::min(batch, k - c0);
    gather(c0, nb, false, E.x[0]);
    solve(h, 0, exact_cfg, E.x[0], E.z[0], nb, &so);
    b_dot(c, h.scratch, h.vec(0, MGM_PREC_F64, E.x[0], nb), h.vec(0, MGM_PREC_F64, E.z[0], nb), E.qf);
    std::vector<double2> q(nb);
    MGM_HIP(hipMemcpyAsync(q.data(), E.qf, sizeof(double2) * nb, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    for (int j = 0; j < nb; j++) tr += std::complex<double>(q[j].x, q[j].y);
  }
  exact = tr;
  exact_seconds = now_s() - t1;
}

}  // namespace mgm
