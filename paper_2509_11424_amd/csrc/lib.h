// Internal objects behind the C ABI: hierarchy, solver workspaces, estimator.
#pragma once
#include "blas.h"
#include "fine.h"
#include "mg.h"
#include "probe.h"

struct mgm_context_s {
  mgm::Context c;
};

struct mgm_operator_s {
  mgm::Context* ctx = nullptr;
  mgm::FineOp op;
  mgm_lattice_desc desc{};
};

namespace mgm {

struct Net;  // learned preconditioner (net.hip)

// Per level and working precision: Krylov basis and V-cycle temporaries.
struct LevelWS {
  mgm_prec prec = MGM_PREC_F64;
  int nmax = 0;  // right-hand sides
  int m = 0;     // restart length
  void* V = nullptr;  // (m+1) vectors
  void* Z = nullptr;  // m vectors (flexible preconditioned directions)
  void* r = nullptr;
  void* t = nullptr;
  void* rho = nullptr;
  void* q = nullptr;
  void* y = nullptr;
  void* bc = nullptr;  // right-hand side of this level's coarse-grid solve
  void* xc = nullptr;  // solution of this level's coarse-grid solve
  Givens G;
  double* n2a = nullptr;   // [nmax] scratch norms
  double* n2b = nullptr;
  double2* qr = nullptr;   // [nmax]
  double* qq = nullptr;
  double2* qr2 = nullptr;  // second pair (fused FP16 smoother: previous step's dots)
  double* qq2 = nullptr;
  double* mask = nullptr;  // [nmax] per-rhs scale factors
};

// FP64 estimator buffers per level, and fine-level term vectors.
struct EstWS {
  int nmax = 0;
  std::vector<double2*> x, y, z, w, u, v;  // per level
  std::vector<double2*> term;             // fine vectors for correlators / loops
  double2* eta = nullptr;                 // fine source (full volume)
  double2* qf = nullptr;                  // [nmax] per-probe values
  double2* qf2 = nullptr;
  double2* slice_partial = nullptr;
  double2* slice_out = nullptr;
};

// test vectors smoothed together in the rough setup recipe
constexpr int kSetupChunk = 4;

// Makes the device of a context current for the duration of one library call
// (and restores the caller's device), so that contexts on different devices
// can be driven from one thread.
struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(const Context* c) {
    if (!c) return;
    int cur = 0;
    MGM_HIP(hipGetDevice(&cur));
    if (cur != c->device) {
      MGM_HIP(hipSetDevice(c->device));
      prev = cur;
    }
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
  DeviceScope(const DeviceScope&) = delete;
  DeviceScope& operator=(const DeviceScope&) = delete;
};

struct Hier {
  Context* ctx = nullptr;
  FineOp* fine = nullptr;
  mgm_hierarchy_desc desc{};
  int L = 0;
  std::vector<LGeom> g;
  std::vector<Transfer> T;
  std::vector<CoarseOp> A;  // A[l] for l >= 1
  Scratch scratch;
  std::vector<LevelWS> ws64, ws32, ws16;
  EstWS est;
  int* d_flag = nullptr;
  double2* dpart = nullptr;  // per-block partial sums of the fused dslash reductions
  double* pinned = nullptr;  // host staging (est, norms)
  size_t pinned_n = 0;
  // setup buffers (alias the solver region)
  std::vector<double2*> tv;  // per transfer: ntv test vectors (FP64)
  double2* setup_v = nullptr;
  double2* setup_y = nullptr;
  double2* setup_rho = nullptr;
  double2* setup_q = nullptr;
  double* setup_n2 = nullptr;
  double2* setup_qr = nullptr;
  double* setup_qq = nullptr;
  bool tv_valid = false;     // test vectors alias solver memory until the first solve
  Net* net = nullptr;
  // captured coarse-grid corrections (level, precision, batch, settings):
  // one eager use, capture on the second, replay afterwards
  struct GraphEntry {
    int uses = 0;
    hipGraphExec_t exec = nullptr;
  };
  std::map<std::string, GraphEntry> graphs;
  ~Hier() {
    for (auto& g : graphs)
      if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
  }

  int64_t n(int l) const { return g[l].V * g[l].dof; }
  // right-hand-side capacity of level l (non-decreasing towards coarse levels)
  int cap(int l) const {
    int c = 0;
    for (int k = 0; k <= l; k++) {
      int v = desc.max_nrhs_level[k] > 0 ? desc.max_nrhs_level[k] : desc.max_nrhs;
      c = std::max(c, v);
    }
    return c;
  }
  Vec vec(int l, mgm_prec p, void* ptr, int nrhs) const {
    Vec v;
    v.p = ptr;
    v.nsite = g[l].V;
    v.dof = g[l].dof;
    v.nrhs = nrhs;
    v.prec = p;
    return v;
  }
  void apply(int l, mgm_prec p, const void* x, void* y, int nrhs) const;
  LevelWS& ws(int l, mgm_prec p) {
    return p == MGM_PREC_F64 ? ws64[l] : p == MGM_PREC_F32 ? ws32[l] : ws16[l];
  }

  void layout(Arena& a);  // carve (or size) every buffer
  void build();           // test vectors, QR, Galerkin, precision copies
  void build_level(int l, const double2* tvsrc);  // transfer l and D_{l+1}
  void rough_tv(int l);                              // rough test vectors of level l into tv[l]
  void finish_level(int l, const double2* src);      // P_l, D_{l+1}, copies from a block of tvs
};

// ------------------------------------------------------------ solver

struct SolveCfg {
  double tol = 1e-10;
  int maxiter = 1000;
  int kind = MGM_SOLVE_MG;
  int smooth = 2;
  int coarse_iters = 12;
  double inner_tol = 1e-5;
  bool coarse_bf16 = false;
  bool smooth_f16 = false;  // mixed kinds: FP16-storage fine MR smoother
  int smooth_coarse = 0;    // MR steps on levels >= 1 (0: smooth)
  bool graphs = false;      // replay captured coarse-grid corrections
  Net* net = nullptr;
};

struct SolveOut {
  int iterations = 0;
  int restarts = 0;
  int fallbacks = 0;
  double max_rel = 0;
  bool converged = true;
};

// Solves D_l x = b (FP64 dof-major) with the configured method.
void solve(Hier& H, int l, const SolveCfg& cfg, const double2* b, double2* x, int nrhs, SolveOut* out);

// e = M r: one V-cycle of level l in precision p (e overwritten)
// unit: every column of r has norm 1 or 0 (a normalised Arnoldi vector)
void vcycle(Hier& H, int l, mgm_prec p, Vec r, Vec e, const SolveCfg& cfg, bool unit = false);

// ------------------------------------------------------------ no-alloc

// Looks up, once per device (with that device current), the device address of
// the fixed scratch array used by mgm_operator_apply_dot_noalloc.
void noalloc_bind_device(int device);

// ------------------------------------------------------------ deflation

constexpr int kStreamDeflBasis = 9;   // Z4 start block of the deflation basis (level 0)
constexpr int kStreamDeflProbe = 10;  // probes of the deflated estimator (level 0)

SolveCfg solve_cfg_of(const mgm_solve_desc* d);

// Inexact deflation basis V (fine level, n x k, orthonormal columns) of a
// hierarchy's fine operator, and tr(V^H D^-1 V).
struct Defl {
  Hier* H = nullptr;
  int k = 0;
  int batch = 0;
  double2* V = nullptr;     // [n][k] dof-major block
  double2* part = nullptr;  // chunk partials of the tall-skinny products
  size_t part_cap = 0;
  double2* C = nullptr;     // [k][max(k, cap0)] product results
  double2* C2 = nullptr;
  double2* M = nullptr;     // [k][k] triangular factor inverse
  std::complex<double> exact = 0.0;
  double setup_seconds = 0, exact_seconds = 0;
  SolveOut so;
  static size_t part_entries(int k, int kb_max);
  void layout(Arena& a);
  void build(const mgm_deflation_desc& d, const SolveCfg& power, const SolveCfg& exact_cfg);
  void cholqr();
  void gather(int c0, int b, bool g5, double2* out);
  void scatter(int c0, int b, const double2* in);
  void vh_times(const double2* X, int nb, double2* out);  // out = V^H X (k x nb)
};

// ------------------------------------------------------------ refinement

size_t refine_workspace_bytes(const Hier& H);
void refine_hierarchy(Hier& H, const mgm_refine_desc& d, const SolveCfg& power, void* ws, size_t ws_bytes,
                      mgm_refine_stats* st, double* rho_out, double* theta_out);

// ------------------------------------------------------------ estimator

void estimate(Hier& H, const mgm_estimate_desc& d, mgm_estimate_result* out);
mgm_estimate_sizes estimate_sizes(const Hier& H, const mgm_estimate_desc& d);

}  // namespace mgm

struct mgm_hierarchy_s {
  mgm::Hier h;
};

struct mgm_deflation_s {
  mgm_hierarchy_s* owner = nullptr;
  mgm::Defl f;
};
