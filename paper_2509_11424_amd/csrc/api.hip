// C ABI of the library: argument checks, status codes, object lifetimes.
#include <cmath>
#include <cstring>

#include "lib.h"
#include "net.h"

using namespace mgm;

namespace mgm {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

void* Context::host_stage(size_t bytes) {
  if (bytes > pinned_bytes) {
    if (pinned) MGM_HIP(hipHostFree(pinned));
    pinned = nullptr;
    MGM_HIP(hipHostMalloc(&pinned, bytes, hipHostMallocDefault));
    pinned_bytes = bytes;
  }
  return pinned;
}

hipEvent_t Context::take_event() {
  if (!prof.pool.empty()) {
    hipEvent_t e = prof.pool.back();
    prof.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  MGM_HIP(hipEventCreate(&e));
  return e;
}

void Context::prof_begin(int, double, hipEvent_t* a) {
  *a = take_event();
  MGM_HIP(hipEventRecord(*a, stream));
}

void Context::prof_end(int kclass, double bytes, hipEvent_t a) {
  hipEvent_t b = take_event();
  MGM_HIP(hipEventRecord(b, stream));
  prof.pending.push_back({a, b, kclass, bytes});
  if (prof.pending.size() > 4096) prof_flush();
}

int Context::choose(const std::string& key, int nvar, const std::function<void(int)>& run, int dflt) {
  auto it = tune.table.find(key);
  if (it != tune.table.end()) {
    MGM_CHECK(it->second.variant < nvar, MGM_ERR_INVALID_ARG,
              "pinned launch variant " + std::to_string(it->second.variant) + " out of range for " + key);
    run(it->second.variant);
    return it->second.variant;
  }
  if (!tune.enabled || capturing || nvar <= 1) {
    run(dflt);
    return dflt;
  }
  const bool prof_was_on = prof.on;
  prof.on = false;  // tuning launches stay out of the kernel-class statistics
  Tuner::Entry e;
  e.ms.assign(nvar, 0.0f);
  hipEvent_t a = take_event(), b = take_event();
  for (int v = 0; v < nvar; v++) {
    run(v);  // warm-up
    float best = 3.0e38f;
    for (int rep = 0; rep < 3; rep++) {
      MGM_HIP(hipEventRecord(a, stream));
      run(v);
      MGM_HIP(hipEventRecord(b, stream));
      MGM_HIP(hipEventSynchronize(b));
      float ms = 0;
      MGM_HIP(hipEventElapsedTime(&ms, a, b));
      best = ms < best ? ms : best;
    }
    e.ms[v] = best;
  }
  int bv = 0;
  for (int v = 1; v < nvar; v++)
    if (e.ms[v] < e.ms[bv]) bv = v;
  e.variant = bv;
  tune.table[key] = e;
  prof.pool.push_back(a);
  prof.pool.push_back(b);
  prof.on = prof_was_on;
  run(bv);  // the call's result comes from the chosen variant
  return bv;
}

void Context::prof_flush() {
  if (prof.pending.empty()) return;
  sync();
  for (auto& r : prof.pending) {
    float ms = 0;
    MGM_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    prof.launches[r.kclass]++;
    prof.ms[r.kclass] += ms;
    prof.bytes[r.kclass] += r.bytes;
    prof.pool.push_back(r.a);
    prof.pool.push_back(r.b);
  }
  prof.pending.clear();
}

}  // namespace mgm

#define API_BEGIN try {
#define API_END                                   \
  return MGM_OK;                                  \
  }                                               \
  catch (const mgm::Error& e) {                   \
    set_last_error(e.what());                     \
    return e.code;                                \
  }                                               \
  catch (const std::exception& e) {               \
    set_last_error(e.what());                     \
    return MGM_ERR_INVALID_ARG;                   \
  }

// the context a handle runs on (nullptr for a NULL handle: the call's own
// argument check reports it)
static const mgm::Context* ctx_of(mgm_context c) { return c ? &c->c : nullptr; }
static const mgm::Context* ctx_of(mgm_operator o) { return o ? o->ctx : nullptr; }
static const mgm::Context* ctx_of(mgm_hierarchy h) { return h ? h->h.ctx : nullptr; }
static const mgm::Context* ctx_of(mgm_deflation f) { return f && f->owner ? f->owner->h.ctx : nullptr; }
static const mgm::Context* ctx_of(mgm_net n) { return n && n->op ? n->op->ctx : nullptr; }
#define API_ON(handle) mgm::DeviceScope device_scope_(ctx_of(handle));

extern "C" {

const char* mgm_status_string(mgm_status s) {
  switch (s) {
    case MGM_OK: return "ok";
    case MGM_ERR_INVALID_ARG: return "invalid argument";
    case MGM_ERR_SHAPE: return "unsupported shape";
    case MGM_ERR_WORKSPACE: return "workspace too small";
    case MGM_ERR_NOT_CONVERGED: return "solver did not converge";
    case MGM_ERR_RANK_DEFICIENT: return "rank-deficient test vectors";
    case MGM_ERR_NUMERIC: return "non-finite value";
    case MGM_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* mgm_last_error(void) { return g_last_error.c_str(); }
const char* mgm_version(void) { return "mgmlmc 0.1 (gfx950)"; }

mgm_status mgm_context_create(int device, void* hip_stream, mgm_context* out) {
  API_BEGIN
  MGM_CHECK(out != nullptr, MGM_ERR_INVALID_ARG, "out is NULL");
  int n = 0;
  MGM_HIP(hipGetDeviceCount(&n));
  MGM_CHECK(device >= 0 && device < n, MGM_ERR_INVALID_ARG, "no such device");
  MGM_HIP(hipSetDevice(device));
  auto* c = new mgm_context_s();
  c->c.device = device;
  c->c.stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  MGM_HIP(hipGetDeviceProperties(&prop, device));
  c->c.cu_count = prop.multiProcessorCount;
  c->c.max_lds = prop.sharedMemPerBlock;
  try {
    noalloc_bind_device(device);  // device address of the allocation-free entry point's scratch
  } catch (...) {
    delete c;
    throw;
  }
  *out = c;
  API_END
}

mgm_status mgm_context_set_stream(mgm_context ctx, void* hip_stream) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx != nullptr, MGM_ERR_INVALID_ARG, "ctx is NULL");
  ctx->c.stream = (hipStream_t)hip_stream;
  API_END
}

mgm_status mgm_context_set_autotune(mgm_context ctx, int32_t enable) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx != nullptr, MGM_ERR_INVALID_ARG, "ctx is NULL");
  ctx->c.tune.enabled = enable != 0;
  API_END
}

mgm_status mgm_context_tune_report(mgm_context ctx, char* buf, size_t bytes, size_t* needed) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx != nullptr, MGM_ERR_INVALID_ARG, "ctx is NULL");
  std::string out;
  for (auto& kv : ctx->c.tune.table) {
    out += kv.first + " " + std::to_string(kv.second.variant);
    for (float ms : kv.second.ms) {
      char t[32];
      std::snprintf(t, sizeof(t), " %.4f", ms);
      out += t;
    }
    out += "\n";
  }
  if (needed) *needed = out.size() + 1;
  if (buf && bytes > 0) {
    const size_t n = std::min(bytes - 1, out.size());
    std::memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  API_END
}

mgm_status mgm_context_tune_set(mgm_context ctx, const char* key, int32_t variant) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx != nullptr && key != nullptr, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(variant >= 0, MGM_ERR_INVALID_ARG, "variant must be >= 0");
  Tuner::Entry e;
  e.variant = variant;
  ctx->c.tune.table[key] = e;
  API_END
}

void mgm_context_destroy(mgm_context ctx) {
  if (!ctx) return;
  try {
    ctx->c.prof_flush();
    for (auto e : ctx->c.prof.pool) (void)hipEventDestroy(e);
    if (ctx->c.pinned) (void)hipHostFree(ctx->c.pinned);
  } catch (...) {
  }
  delete ctx;
}

// ------------------------------------------------------------ operator

static Geom geom_of(const mgm_lattice_desc* d) {
  MGM_CHECK(d != nullptr, MGM_ERR_INVALID_ARG, "desc is NULL");
  for (int m = 0; m < 4; m++) MGM_CHECK(d->dims[m] >= 2, MGM_ERR_SHAPE, "every lattice extent must be >= 2");
  MGM_CHECK(std::isfinite(d->m0) && std::isfinite(d->csw), MGM_ERR_INVALID_ARG, "non-finite m0 or csw");
  Geom g;
  g.X = d->dims[0];
  g.Y = d->dims[1];
  g.Z = d->dims[2];
  g.T = d->dims[3];
  g.V = (int64_t)g.X * g.Y * g.Z * g.T;
  g.antiperiodic = d->t_antiperiodic ? 1 : 0;
  return g;
}

mgm_status mgm_operator_workspace_size(const mgm_lattice_desc* desc, size_t* bytes) {
  API_BEGIN
  MGM_CHECK(bytes != nullptr, MGM_ERR_INVALID_ARG, "bytes is NULL");
  Geom g = geom_of(desc);
  Arena a;
  FineOp tmp;
  FineOp::layout(a, g, &tmp);
  *bytes = a.off;
  API_END
}

mgm_status mgm_operator_create(mgm_context ctx, const mgm_lattice_desc* desc, const double* gauge_host,
                               void* ws_dev, size_t ws_bytes, mgm_operator* out) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx && gauge_host && ws_dev && out, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(((uintptr_t)ws_dev & 255) == 0, MGM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  Geom g = geom_of(desc);
  Arena a;
  a.base = (char*)ws_dev;
  a.cap = ws_bytes;
  auto* op = new mgm_operator_s();
  try {
    op->ctx = &ctx->c;
    op->desc = *desc;
    op->op.ctx = &ctx->c;
    op->op.m0 = desc->m0;
    op->op.csw = desc->csw;
    FineOp::layout(a, g, &op->op);
    op->op.build(gauge_host);
  } catch (...) {
    delete op;
    throw;
  }
  *out = op;
  API_END
}

mgm_status mgm_operator_apply(mgm_operator op, mgm_prec prec, const void* x, void* y, int32_t nrhs) {
  API_BEGIN
  API_ON(op)
  MGM_CHECK(op && x && y && nrhs >= 1, MGM_ERR_INVALID_ARG, "bad arguments");
  MGM_CHECK(x != y, MGM_ERR_INVALID_ARG, "x and y must not overlap");
  op->op.apply(prec, x, y, nrhs);
  API_END
}

static size_t dot_ws_bytes(const FineOp& op, mgm_prec prec, int nrhs) {
  // block partials [2][nrhs][blocks] plus the segment sums of the finalisation
  return ((size_t)op.nblocks(prec, nrhs, true) * 2 * nrhs + (size_t)64 * 2 * nrhs) * sizeof(double2) + 256;
}

mgm_status mgm_operator_dot_workspace_size(mgm_operator op, mgm_prec prec, int32_t nrhs, size_t* bytes) {
  API_BEGIN
  API_ON(op)
  MGM_CHECK(op && bytes && nrhs >= 1 && nrhs <= 256, MGM_ERR_INVALID_ARG, "bad arguments");
  *bytes = dot_ws_bytes(op->op, prec, nrhs);
  API_END
}

mgm_status mgm_operator_apply_dot(mgm_operator op, mgm_prec prec, const void* x, void* y, int32_t nrhs,
                                  void* ws_dev, size_t ws_bytes, void* yx_dev, void* yy_dev) {
  API_BEGIN
  API_ON(op)
  MGM_CHECK(op && x && y && ws_dev && yx_dev && yy_dev, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(nrhs >= 1 && nrhs <= 256, MGM_ERR_INVALID_ARG, "nrhs must be 1..256");
  MGM_CHECK(x != y, MGM_ERR_INVALID_ARG, "x and y must not overlap");
  MGM_CHECK(((uintptr_t)ws_dev & 255) == 0, MGM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  MGM_CHECK(ws_bytes >= dot_ws_bytes(op->op, prec, nrhs), MGM_ERR_WORKSPACE, "dot workspace too small");
  const int64_t nb = op->op.nblocks(prec, nrhs, true);
  double2* part = (double2*)ws_dev;
  Scratch sc;
  sc.partial = part + (size_t)nb * 2 * nrhs;
  sc.cap = (size_t)64 * 2 * nrhs;
  const int64_t nrun = op->op.apply_dot(prec, x, y, nrhs, part);
  b_finalize_dot_norm(op->ctx, sc, part, nrun, nrhs, (double2*)yx_dev, (double*)yy_dev);
  API_END
}

mgm_status mgm_operator_smoother_step(mgm_operator op, const void* r_dev, void* r_next_dev, void* x_dev,
                                      const void* qr_prev_dev, const void* qq_prev_dev, int32_t nrhs,
                                      void* ws_dev, size_t ws_bytes, void* yx_dev, void* yy_dev) {
  API_BEGIN
  API_ON(op)
  MGM_CHECK(op && r_dev && r_next_dev && x_dev && qr_prev_dev && qq_prev_dev && ws_dev && yx_dev && yy_dev,
            MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(nrhs >= 1 && nrhs <= 256, MGM_ERR_INVALID_ARG, "nrhs must be 1..256");
  MGM_CHECK(((uintptr_t)ws_dev & 255) == 0, MGM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  MGM_CHECK(ws_bytes >= dot_ws_bytes(op->op, MGM_PREC_F16, nrhs), MGM_ERR_WORKSPACE, "workspace too small");
  MGM_CHECK(op->op.step_fusable(MGM_PREC_F16, nrhs), MGM_ERR_SHAPE, "no plane-marching tile for this lattice and nrhs");
  const int64_t nb = op->op.nblocks(MGM_PREC_F16, nrhs, true);
  double2* part = (double2*)ws_dev;
  Scratch sc;
  sc.partial = part + (size_t)nb * 2 * nrhs;
  sc.cap = (size_t)64 * 2 * nrhs;
  const int64_t nrun = op->op.apply_step(MGM_PREC_F16, r_dev, r_next_dev, x_dev, (const double2*)qr_prev_dev,
                                         (const double*)qq_prev_dev, nrhs, part);
  b_finalize_dot_norm(op->ctx, sc, part, nrun, nrhs, (double2*)yx_dev, (double*)yy_dev);
  API_END
}

int32_t mgm_operator_step_fusable(mgm_operator op, int32_t nrhs) {
  if (!op || nrhs < 1 || nrhs > 256) return 0;
  try {
    return op->op.step_fusable(MGM_PREC_F16, nrhs) ? 1 : 0;
  } catch (...) {
    return 0;
  }
}

int64_t mgm_operator_sites(mgm_operator op) { return op ? op->op.g.V : 0; }
void mgm_operator_destroy(mgm_operator op) { delete op; }

// --------------------------------------------------------------- probes

mgm_status mgm_draw_noise(mgm_context ctx, int32_t kind, uint64_t seed, uint32_t stream, uint64_t first_probe,
                          int32_t nprobe, int64_t n_site, int32_t dof, mgm_prec prec, void* out_dev) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx && out_dev && nprobe >= 1 && n_site >= 1 && dof >= 1, MGM_ERR_INVALID_ARG, "bad arguments");
  MGM_CHECK(first_probe + (uint64_t)nprobe <= (1ull << 32), MGM_ERR_INVALID_ARG,
            "probe indices must be below 2^32 (32-bit counter word)");
  NoiseMask mk;
  draw_noise(&ctx->c, kind, seed, stream, first_probe, nprobe, n_site, dof, prec, out_dev, mk);
  API_END
}

mgm_status mgm_draw_z4(mgm_context ctx, uint64_t seed, uint32_t stream, uint64_t first_probe, int32_t nprobe,
                       int64_t n_site, int32_t dof, mgm_prec prec, void* out) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx && out && nprobe >= 1 && n_site >= 1 && dof >= 1, MGM_ERR_INVALID_ARG, "bad arguments");
  MGM_CHECK(first_probe + (uint64_t)nprobe <= (1ull << 32), MGM_ERR_INVALID_ARG,
            "probe indices must be below 2^32 (32-bit counter word)");
  draw_z4(&ctx->c, seed, stream, first_probe, nprobe, n_site, dof, prec, out);
  API_END
}

// ------------------------------------------------------------ hierarchy

static void check_hdesc(mgm_operator op, const mgm_hierarchy_desc* d) {
  MGM_CHECK(op && d, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(d->nlevels >= 2 && d->nlevels <= MGM_MAX_LEVELS, MGM_ERR_INVALID_ARG, "nlevels must be 2..4");
  MGM_CHECK(d->setup_steps >= 1 && d->setup_mr >= 1, MGM_ERR_INVALID_ARG, "setup steps must be >= 1");
  MGM_CHECK(d->max_nrhs >= 1 && d->max_nrhs <= 256, MGM_ERR_INVALID_ARG, "max_nrhs must be 1..256");
  for (int l = 0; l < MGM_MAX_LEVELS; l++)
    MGM_CHECK(d->max_nrhs_level[l] >= 0 && d->max_nrhs_level[l] <= 256, MGM_ERR_INVALID_ARG,
              "max_nrhs_level must be 0..256");
  MGM_CHECK(d->restart >= 2 && d->restart <= 63, MGM_ERR_INVALID_ARG, "restart must be 2..63");
  int dims[4] = {op->op.g.X, op->op.g.Y, op->op.g.Z, op->op.g.T};
  int dof = 12;
  for (int l = 0; l + 1 < d->nlevels; l++) {
    MGM_CHECK(d->ntv[l] >= 1 && d->ntv[l] <= 128, MGM_ERR_INVALID_ARG, "ntv must be 1..128");
    MGM_CHECK(2 * d->ntv[l] <= 256 && dof <= 256, MGM_ERR_SHAPE, "coarse dof must be <= 256");
    for (int m = 0; m < 4; m++) {
      int b = d->block[l][m];
      MGM_CHECK(b >= 1 && dims[m] % b == 0 && dims[m] / b >= 2, MGM_ERR_SHAPE,
                "lattice not divisible into aggregates with coarse extent >= 2");
      dims[m] /= b;
    }
    const int bvol = d->block[l][0] * d->block[l][1] * d->block[l][2] * d->block[l][3];
    int rows = bvol * (dof / 2);
    MGM_CHECK(rows * 16 <= 64 * 1024 && bvol <= 1024, MGM_ERR_SHAPE, "aggregate too large");
    MGM_CHECK(d->ntv[l] <= rows, MGM_ERR_RANK_DEFICIENT, "more test vectors than aggregate rows");
    dof = 2 * d->ntv[l];
  }
}

mgm_status mgm_hierarchy_workspace_size(mgm_operator op, const mgm_hierarchy_desc* desc, size_t* bytes) {
  API_BEGIN
  API_ON(op)
  check_hdesc(op, desc);
  MGM_CHECK(bytes, MGM_ERR_INVALID_ARG, "bytes is NULL");
  Hier h;
  h.ctx = op->ctx;
  h.fine = &op->op;
  h.desc = *desc;
  Arena a;
  h.layout(a);
  *bytes = a.off;
  API_END
}

mgm_status mgm_hierarchy_create(mgm_operator op, const mgm_hierarchy_desc* desc, void* ws_dev, size_t ws_bytes,
                                mgm_hierarchy* out) {
  API_BEGIN
  API_ON(op)
  check_hdesc(op, desc);
  MGM_CHECK(ws_dev && out, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(((uintptr_t)ws_dev & 255) == 0, MGM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  auto* hh = new mgm_hierarchy_s();
  try {
    Hier& h = hh->h;
    h.ctx = op->ctx;
    h.fine = &op->op;
    h.desc = *desc;
    Arena a;
    a.base = (char*)ws_dev;
    a.cap = ws_bytes;
    h.layout(a);
    h.pinned_n = 4 * 256;
    h.pinned = (double*)h.ctx->host_stage(h.pinned_n * sizeof(double));
    h.build();
    h.tv_valid = true;
  } catch (...) {
    delete hh;
    throw;
  }
  *out = hh;
  API_END
}

mgm_status mgm_hierarchy_level_info(mgm_hierarchy h, int32_t level, int64_t* sites, int32_t* dof, int64_t* n) {
  API_BEGIN
  API_ON(h)
  MGM_CHECK(h && level >= 0 && level < h->h.L, MGM_ERR_INVALID_ARG, "bad level");
  if (sites) *sites = h->h.g[level].V;
  if (dof) *dof = h->h.g[level].dof;
  if (n) *n = h->h.n(level);
  API_END
}

mgm_status mgm_hierarchy_export(mgm_hierarchy hh, int32_t level, mgm_export_kind what, void* host_buf,
                                size_t bytes) {
  API_BEGIN
  API_ON(hh)
  MGM_CHECK(hh && host_buf, MGM_ERR_INVALID_ARG, "NULL argument");
  Hier& h = hh->h;
  MGM_CHECK(level >= 0 && level + 1 < h.L, MGM_ERR_INVALID_ARG, "bad transfer level");
  Context* c = h.ctx;
  const TGeom& t = h.T[level].t;
  if (what == MGM_EXPORT_AGG_MAP) {
    size_t need = (size_t)t.c.V * 2 * t.rows * sizeof(int64_t);
    MGM_CHECK(bytes >= need, MGM_ERR_INVALID_ARG, "buffer too small");
    MGM_CHECK(h.ws64[level].prec == MGM_PREC_F64 && h.ws64[level].r, MGM_ERR_WORKSPACE, "no scratch");
    h.tv_valid = false;
    int64_t* tmp = (int64_t*)h.ws64[level].r;  // scratch: n_l * nmax * 16 bytes >= n_l * 8
    mg_agg_map(c, t, tmp);
    MGM_HIP(hipMemcpyAsync(host_buf, tmp, need, hipMemcpyDeviceToHost, c->stream));
    c->sync();
  } else if (what == MGM_EXPORT_P) {
    size_t need = (size_t)t.c.V * 2 * t.rows * t.ntv * sizeof(double2);
    MGM_CHECK(bytes >= need, MGM_ERR_INVALID_ARG, "buffer too small");
    MGM_HIP(hipMemcpyAsync(host_buf, h.T[level].P64, need, hipMemcpyDeviceToHost, c->stream));
    c->sync();
  } else if (what == MGM_EXPORT_COARSE) {
    const CoarseOp& A = h.A[level + 1];
    const int d = A.d;
    const int64_t V = A.g.V;
    size_t need = (size_t)V * 9 * d * d * sizeof(double2);
    MGM_CHECK(bytes >= need, MGM_ERR_INVALID_ARG, "buffer too small");
    std::vector<double2> tmp((size_t)V * 9 * d * d);
    MGM_HIP(hipMemcpyAsync(tmp.data(), A.A64, need, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    double2* o = (double2*)host_buf;
    for (int k = 0; k < 9; k++)
      for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++)
          for (int64_t s = 0; s < V; s++)
            o[((s * 9 + k) * d + i) * d + j] = tmp[(((size_t)k * d + i) * d + j) * V + s];
  } else if (what == MGM_EXPORT_TV) {
    MGM_CHECK(h.tv_valid, MGM_ERR_INVALID_ARG, "test vectors are only kept until the first solve");
    const int ntv = t.ntv;
    const int64_t nl = h.n(level);
    size_t need = (size_t)ntv * nl * sizeof(double2);
    MGM_CHECK(bytes >= need, MGM_ERR_INVALID_ARG, "buffer too small");
    std::vector<double2> tmp((size_t)ntv * nl);
    MGM_HIP(hipMemcpyAsync(tmp.data(), h.tv[level], need, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    // dof-major [dof][site][k] -> [k][site*dof + dof]
    const int dof = h.g[level].dof;
    const int64_t V = h.g[level].V;
    double2* o = (double2*)host_buf;
    for (int dd = 0; dd < dof; dd++)
      for (int64_t s = 0; s < V; s++)
        for (int k = 0; k < ntv; k++) o[(size_t)k * nl + s * dof + dd] = tmp[((size_t)dd * V + s) * ntv + k];
  } else {
    throw Error(MGM_ERR_INVALID_ARG, "unknown export kind");
  }
  API_END
}

static void check_level(mgm_hierarchy h, int level, int nrhs, bool transfer) {
  MGM_CHECK(h != nullptr, MGM_ERR_INVALID_ARG, "h is NULL");
  MGM_CHECK(level >= 0 && level < h->h.L - (transfer ? 1 : 0), MGM_ERR_INVALID_ARG, "bad level");
  MGM_CHECK(nrhs >= 1, MGM_ERR_INVALID_ARG, "nrhs must be >= 1");
}

mgm_status mgm_level_apply(mgm_hierarchy h, int32_t level, const void* x, void* y, int32_t nrhs) {
  API_BEGIN
  API_ON(h)
  check_level(h, level, nrhs, false);
  MGM_CHECK(x && y && x != y, MGM_ERR_INVALID_ARG, "bad vectors");
  h->h.apply(level, MGM_PREC_F64, x, y, nrhs);
  API_END
}

mgm_status mgm_level_apply_prec(mgm_hierarchy h, int32_t level, mgm_prec prec, const void* x, void* y,
                                int32_t nrhs) {
  API_BEGIN
  API_ON(h)
  check_level(h, level, nrhs, false);
  MGM_CHECK(x && y && x != y, MGM_ERR_INVALID_ARG, "bad vectors");
  MGM_CHECK(!(level == 0 && prec == MGM_PREC_BF16) && !(level > 0 && prec == MGM_PREC_F16), MGM_ERR_INVALID_ARG,
            "F16 exists on the fine level, BF16 on coarse levels");
  h->h.apply(level, prec, x, y, nrhs);
  API_END
}

mgm_status mgm_restrict(mgm_hierarchy h, int32_t level, const void* x, void* y, int32_t nrhs) {
  API_BEGIN
  API_ON(h)
  check_level(h, level, nrhs, true);
  MGM_CHECK(x && y, MGM_ERR_INVALID_ARG, "bad vectors");
  h->h.T[level].restrict_(MGM_PREC_F64, x, y, nrhs);
  API_END
}

mgm_status mgm_prolong(mgm_hierarchy h, int32_t level, const void* x, void* y, int32_t nrhs) {
  API_BEGIN
  API_ON(h)
  check_level(h, level, nrhs, true);
  MGM_CHECK(x && y, MGM_ERR_INVALID_ARG, "bad vectors");
  h->h.T[level].prolong(MGM_PREC_F64, x, nullptr, y, nrhs, 0);
  API_END
}

static void check_transfer_prec(mgm_hierarchy h, mgm_prec prec) {
  MGM_CHECK(prec == MGM_PREC_F64 || prec == MGM_PREC_F32, MGM_ERR_INVALID_ARG,
            "transfers run in F64 or F32");
  MGM_CHECK(prec == MGM_PREC_F64 || h->h.desc.mixed, MGM_ERR_INVALID_ARG,
            "F32 transfers need a hierarchy built with mixed != 0");
}

mgm_status mgm_restrict_prec(mgm_hierarchy h, int32_t level, mgm_prec prec, const void* x, void* y,
                             int32_t nrhs) {
  API_BEGIN
  API_ON(h)
  check_level(h, level, nrhs, true);
  MGM_CHECK(x && y, MGM_ERR_INVALID_ARG, "bad vectors");
  check_transfer_prec(h, prec);
  h->h.T[level].restrict_(prec, x, y, nrhs);
  API_END
}

mgm_status mgm_prolong_prec(mgm_hierarchy h, int32_t level, mgm_prec prec, const void* x, void* y,
                            int32_t nrhs) {
  API_BEGIN
  API_ON(h)
  check_level(h, level, nrhs, true);
  MGM_CHECK(x && y, MGM_ERR_INVALID_ARG, "bad vectors");
  check_transfer_prec(h, prec);
  h->h.T[level].prolong(prec, x, nullptr, y, nrhs, 0);
  API_END
}

mgm_status mgm_restrict_f16(mgm_hierarchy h, int32_t level, const void* x16, const double* scale, void* y,
                            int32_t nrhs) {
  API_BEGIN
  API_ON(h)
  check_level(h, level, nrhs, true);
  MGM_CHECK(x16 && scale && y && x16 != y, MGM_ERR_INVALID_ARG, "bad vectors");
  check_transfer_prec(h, MGM_PREC_F32);
  h->h.T[level].restrict16((const __half2*)x16, scale, (float2*)y, nrhs);
  API_END
}

mgm_status mgm_prolong_add_f16(mgm_hierarchy h, int32_t level, const void* xc, const void* x16,
                               const double* scale, void* y, int32_t nrhs) {
  API_BEGIN
  API_ON(h)
  check_level(h, level, nrhs, true);
  MGM_CHECK(xc && x16 && scale && y && y != x16 && y != xc, MGM_ERR_INVALID_ARG, "bad vectors");
  check_transfer_prec(h, MGM_PREC_F32);
  h->h.T[level].prolong16((const float2*)xc, (const __half2*)x16, scale, (float2*)y, nrhs);
  API_END
}

mgm_status mgm_project_out(mgm_hierarchy h, int32_t level, const void* x, void* y, int32_t nrhs) {
  API_BEGIN
  API_ON(h)
  check_level(h, level, nrhs, true);
  MGM_CHECK(x && y, MGM_ERR_INVALID_ARG, "bad vectors");
  Hier& H = h->h;
  MGM_CHECK(nrhs <= H.cap(level), MGM_ERR_INVALID_ARG, "nrhs exceeds the capacity of the level");
  H.T[level].restrict_(MGM_PREC_F64, x, H.est.w[level + 1], nrhs);
  H.T[level].prolong(MGM_PREC_F64, H.est.w[level + 1], x, y, nrhs, 1);
  API_END
}

static SolveCfg cfg_of(const mgm_solve_desc* d) {
  MGM_CHECK(d != nullptr, MGM_ERR_INVALID_ARG, "solve desc is NULL");
  MGM_CHECK(d->tol > 0 && d->maxiter >= 1 && d->smooth >= 0 && d->smooth_coarse >= 0 && d->coarse_iters >= 1,
            MGM_ERR_INVALID_ARG,
            "bad solve parameters");
  SolveCfg c;
  c.tol = d->tol;
  c.maxiter = d->maxiter;
  c.kind = d->kind;
  c.smooth = d->smooth;
  c.smooth_coarse = d->smooth_coarse;
  c.coarse_iters = d->coarse_iters;
  c.inner_tol = d->inner_tol > 0 ? d->inner_tol : 1e-5;
  c.coarse_bf16 = d->coarse_bf16 != 0;
  c.smooth_f16 = d->smoother_f16 != 0;
  c.graphs = d->graphs != 0;
  c.net = (Net*)d->net;
  MGM_CHECK(c.kind != MGM_SOLVE_NET || c.net != nullptr, MGM_ERR_INVALID_ARG, "NET solve needs a network");
  return c;
}

mgm_status mgm_solve(mgm_hierarchy h, int32_t level, const mgm_solve_desc* desc, const void* b, void* x,
                     int32_t nrhs, mgm_solve_stats* stats) {
  mgm_status st = MGM_OK;
  try {
    API_ON(h)
    check_level(h, level, nrhs, false);
    MGM_CHECK(b && x && b != x, MGM_ERR_INVALID_ARG, "bad vectors");
    SolveCfg cfg = cfg_of(desc);
    SolveOut out;
    auto t0 = std::chrono::steady_clock::now();
    solve(h->h, level, cfg, (const double2*)b, (double2*)x, nrhs, &out);
    double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) {
      stats->iterations = out.iterations;
      stats->restarts = out.restarts;
      stats->fallbacks = out.fallbacks;
      stats->max_rel_residual = out.max_rel;
      stats->seconds = dt;
    }
    if (!out.converged) {
      set_last_error("solve did not reach the tolerance");
      st = MGM_ERR_NOT_CONVERGED;
    }
  } catch (const mgm::Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return MGM_ERR_INVALID_ARG;
  }
  return st;
}

mgm_status mgm_estimate_sizes_query(mgm_hierarchy h, const mgm_estimate_desc* desc, mgm_estimate_sizes* sizes) {
  API_BEGIN
  API_ON(h)
  MGM_CHECK(h && desc && sizes, MGM_ERR_INVALID_ARG, "NULL argument");
  *sizes = estimate_sizes(h->h, *desc);
  API_END
}

mgm_status mgm_estimate(mgm_hierarchy h, const mgm_estimate_desc* desc, mgm_estimate_result* out) {
  API_BEGIN
  API_ON(h)
  MGM_CHECK(h && desc && out, MGM_ERR_INVALID_ARG, "NULL argument");
  cfg_of(&desc->solve);
  auto t0 = std::chrono::steady_clock::now();
  estimate(h->h, *desc, out);
  out->stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  API_END
}

// ----------------------------------------------------------- refinement

mgm_status mgm_hierarchy_refine_workspace_size(mgm_hierarchy h, size_t* bytes) {
  API_BEGIN
  API_ON(h)
  MGM_CHECK(h && bytes, MGM_ERR_INVALID_ARG, "NULL argument");
  *bytes = refine_workspace_bytes(h->h);
  API_END
}

mgm_status mgm_hierarchy_refine(mgm_hierarchy h, const mgm_refine_desc* desc, void* ws_dev, size_t ws_bytes,
                                mgm_refine_stats* stats, double* rho_host, double* theta_host) {
  API_BEGIN
  API_ON(h)
  MGM_CHECK(h && desc && ws_dev, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(((uintptr_t)ws_dev & 255) == 0, MGM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  MGM_CHECK(ws_bytes >= refine_workspace_bytes(h->h), MGM_ERR_WORKSPACE, "refinement workspace too small");
  MGM_CHECK(desc->max_iters >= 0 && desc->eig_tol >= 0 && desc->power_tol > 0, MGM_ERR_INVALID_ARG,
            "bad refinement settings");
  MGM_CHECK(desc->batch >= 1 && desc->batch <= h->h.cap(0), MGM_ERR_INVALID_ARG,
            "refinement batch must be 1..the fine-level capacity");
  MGM_CHECK(h->h.L >= 2, MGM_ERR_INVALID_ARG, "the hierarchy has no transfer to refine");
  SolveCfg power = cfg_of(&desc->solve);
  power.tol = desc->power_tol;
  refine_hierarchy(h->h, *desc, power, ws_dev, ws_bytes, stats, rho_host, theta_host);
  API_END
}

// ------------------------------------------------------------ deflation

static void check_defl_desc(mgm_hierarchy h, const mgm_deflation_desc* d) {
  MGM_CHECK(h && d, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(d->k >= 1 && d->k <= 1024, MGM_ERR_INVALID_ARG, "deflation basis size must be 1..1024");
  MGM_CHECK(d->k <= h->h.n(0), MGM_ERR_INVALID_ARG, "deflation basis larger than the fine dimension");
  MGM_CHECK(d->power_iters >= 0 && d->power_tol > 0, MGM_ERR_INVALID_ARG, "bad power-step settings");
  MGM_CHECK(d->batch >= 1 && d->batch <= h->h.cap(0), MGM_ERR_INVALID_ARG,
            "deflation batch must be 1..the fine-level capacity");
}

mgm_status mgm_deflation_workspace_size(mgm_hierarchy h, const mgm_deflation_desc* desc, size_t* bytes) {
  API_BEGIN
  API_ON(h)
  check_defl_desc(h, desc);
  MGM_CHECK(bytes != nullptr, MGM_ERR_INVALID_ARG, "bytes is NULL");
  Defl f;
  f.H = &h->h;
  f.k = desc->k;
  Arena a;
  f.layout(a);
  *bytes = a.off;
  API_END
}

mgm_status mgm_deflation_create(mgm_hierarchy h, const mgm_deflation_desc* desc, void* ws_dev, size_t ws_bytes,
                                mgm_deflation* out) {
  mgm_status st = MGM_OK;
  try {
    API_ON(h)
    check_defl_desc(h, desc);
    MGM_CHECK(ws_dev && out, MGM_ERR_INVALID_ARG, "NULL argument");
    MGM_CHECK(((uintptr_t)ws_dev & 255) == 0, MGM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    SolveCfg power = cfg_of(&desc->solve);
    SolveCfg exact = power;
    power.tol = desc->power_tol;
    auto* f = new mgm_deflation_s();
    try {
      f->owner = h;
      f->f.H = &h->h;
      f->f.k = desc->k;
      f->f.batch = desc->batch;
      Arena a;
      a.base = (char*)ws_dev;
      a.cap = ws_bytes;
      f->f.layout(a);
      f->f.build(*desc, power, exact);
    } catch (...) {
      delete f;
      throw;
    }
    *out = f;
    if (!f->f.so.converged) {
      set_last_error("a deflation solve did not reach its tolerance");
      st = MGM_ERR_NOT_CONVERGED;
    }
  } catch (const mgm::Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return MGM_ERR_INVALID_ARG;
  }
  return st;
}

mgm_status mgm_deflation_export(mgm_deflation f, double* host_buf, size_t bytes) {
  API_BEGIN
  API_ON(f)
  MGM_CHECK(f && host_buf, MGM_ERR_INVALID_ARG, "NULL argument");
  const size_t need = (size_t)f->f.H->n(0) * f->f.k * sizeof(double2);
  MGM_CHECK(bytes >= need, MGM_ERR_INVALID_ARG, "host buffer too small");
  Context* c = f->f.H->ctx;
  MGM_HIP(hipMemcpyAsync(host_buf, f->f.V, need, hipMemcpyDeviceToHost, c->stream));
  c->sync();
  API_END
}

mgm_status mgm_deflation_info(mgm_deflation f, double* exact_trace, double* setup_s, double* exact_s) {
  API_BEGIN
  API_ON(f)
  MGM_CHECK(f != nullptr, MGM_ERR_INVALID_ARG, "NULL argument");
  if (exact_trace) {
    exact_trace[0] = f->f.exact.real();
    exact_trace[1] = f->f.exact.imag();
  }
  if (setup_s) *setup_s = f->f.setup_seconds;
  if (exact_s) *exact_s = f->f.exact_seconds;
  API_END
}

void mgm_deflation_destroy(mgm_deflation f) { delete f; }

mgm_status mgm_mlmc_allocate(int32_t nterms, const double* var, const double* cost, double eps2, int64_t* n_out) {
  API_BEGIN
  MGM_CHECK(nterms >= 1 && var && cost && n_out && eps2 > 0, MGM_ERR_INVALID_ARG, "bad arguments");
  double s = 0;
  for (int i = 0; i < nterms; i++) {
    MGM_CHECK(var[i] >= 0 && cost[i] > 0, MGM_ERR_INVALID_ARG, "variances >= 0 and costs > 0 required");
    s += std::sqrt(var[i] * cost[i]);
  }
  for (int i = 0; i < nterms; i++) {
    double n = std::sqrt(var[i] / cost[i]) * s / eps2;
    int64_t k = (int64_t)std::ceil(n);
    n_out[i] = k < 2 ? 2 : k;
  }
  API_END
}

mgm_status mgm_profile_enable(mgm_context ctx, int32_t on) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx, MGM_ERR_INVALID_ARG, "ctx is NULL");
  ctx->c.prof.on = on != 0;
  API_END
}

mgm_status mgm_profile_reset(mgm_context ctx) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx, MGM_ERR_INVALID_ARG, "ctx is NULL");
  ctx->c.prof_flush();
  for (int k = 0; k < KC_COUNT; k++) {
    ctx->c.prof.launches[k] = 0;
    ctx->c.prof.ms[k] = 0;
    ctx->c.prof.bytes[k] = 0;
  }
  API_END
}

mgm_status mgm_profile_query(mgm_context ctx, int32_t kclass, int64_t* launches, double* ms, double* bytes) {
  API_BEGIN
  API_ON(ctx)
  MGM_CHECK(ctx && kclass >= 0 && kclass < KC_COUNT, MGM_ERR_INVALID_ARG, "bad arguments");
  ctx->c.prof_flush();
  if (launches) *launches = ctx->c.prof.launches[kclass];
  if (ms) *ms = ctx->c.prof.ms[kclass];
  if (bytes) *bytes = ctx->c.prof.bytes[kclass];
  API_END
}

void mgm_hierarchy_destroy(mgm_hierarchy h) { delete h; }

// -------------------------------------------------------------- network

static void check_net_desc(mgm_operator op, const mgm_net_desc* d) {
  MGM_CHECK(op != nullptr && d != nullptr, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(d->nlayers >= 1 && d->nlayers <= MGM_NET_MAX_LAYERS, MGM_ERR_INVALID_ARG, "nlayers must be 1..8");
  MGM_CHECK(d->width[0] == 4 && d->width[d->nlayers] == 4, MGM_ERR_INVALID_ARG,
            "the network maps spinors to spinors: width[0] = width[nlayers] = 4");
  for (int l = 0; l <= d->nlayers; l++) {
    const int w = d->width[l];
    MGM_CHECK(w == 4 || w == 8 || w == 12 || w == 16, MGM_ERR_INVALID_ARG, "widths must be 4, 8, 12 or 16");
  }
  MGM_CHECK(d->max_nrhs >= 1 && d->max_nrhs <= 256, MGM_ERR_INVALID_ARG, "max_nrhs must be 1..256");
  MGM_CHECK(d->train_nrhs >= 0 && d->train_nrhs <= 256, MGM_ERR_INVALID_ARG, "train_nrhs must be 0..256");
}

mgm_status mgm_net_workspace_size(mgm_operator op, const mgm_net_desc* desc, size_t* bytes) {
  API_BEGIN
  API_ON(op)
  check_net_desc(op, desc);
  MGM_CHECK(bytes != nullptr, MGM_ERR_INVALID_ARG, "bytes is NULL");
  Net n;
  n.op = &op->op;
  n.desc = *desc;
  Arena a;
  n.layout(a);
  *bytes = a.off;
  API_END
}

mgm_status mgm_net_create(mgm_operator op, const mgm_net_desc* desc, void* ws_dev, size_t ws_bytes,
                          mgm_net* out) {
  API_BEGIN
  API_ON(op)
  check_net_desc(op, desc);
  MGM_CHECK(ws_dev && out, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_CHECK(((uintptr_t)ws_dev & 255) == 0, MGM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  auto* h = new mgm_net_s();
  try {
    h->op = op;
    Net& n = h->n;
    n.ctx = op->ctx;
    n.op = &op->op;
    n.desc = *desc;
    Arena a;
    a.base = (char*)ws_dev;
    a.cap = ws_bytes;
    n.layout(a);
    MGM_HIP(hipHostMalloc((void**)&n.pinned, 64 * sizeof(double), hipHostMallocDefault));
    n.upload_weights(net_initial_weights(n, desc->seed));
  } catch (...) {
    if (h->n.pinned) (void)hipHostFree(h->n.pinned);
    delete h;
    throw;
  }
  *out = h;
  API_END
}

mgm_status mgm_net_bind(mgm_net net, mgm_operator op) {
  API_BEGIN
  API_ON(net)
  MGM_CHECK(net && op, MGM_ERR_INVALID_ARG, "NULL argument");
  const Geom& a = net->n.op->g;
  const Geom& b = op->op.g;
  MGM_CHECK(a.X == b.X && a.Y == b.Y && a.Z == b.Z && a.T == b.T && a.antiperiodic == b.antiperiodic,
            MGM_ERR_SHAPE, "the network can only move to an operator of the same lattice");
  MGM_CHECK(op->ctx == net->n.ctx, MGM_ERR_INVALID_ARG, "the operator belongs to another context");
  net->op = op;
  net->n.op = &op->op;
  API_END
}

mgm_status mgm_net_num_weights(mgm_net net, int64_t* count) {
  API_BEGIN
  API_ON(net)
  MGM_CHECK(net && count, MGM_ERR_INVALID_ARG, "NULL argument");
  *count = net->n.nw;
  API_END
}

mgm_status mgm_net_set_weights(mgm_net net, const double* w_host) {
  API_BEGIN
  API_ON(net)
  MGM_CHECK(net && w_host, MGM_ERR_INVALID_ARG, "NULL argument");
  std::vector<double> w(w_host, w_host + 2 * net->n.nw);
  net->n.upload_weights(w);
  API_END
}

mgm_status mgm_net_get_weights(mgm_net net, double* w_host) {
  API_BEGIN
  API_ON(net)
  MGM_CHECK(net && w_host, MGM_ERR_INVALID_ARG, "NULL argument");
  MGM_HIP(hipMemcpyAsync(w_host, net->n.w64, sizeof(double2) * net->n.nw, hipMemcpyDeviceToHost,
                         net->n.ctx->stream));
  net->n.ctx->sync();
  API_END
}

static const char kNetMagic[8] = {'M', 'G', 'M', 'N', 'E', 'T', '0', '1'};

mgm_status mgm_net_save(mgm_net net, const char* path) {
  API_BEGIN
  API_ON(net)
  MGM_CHECK(net && path, MGM_ERR_INVALID_ARG, "NULL argument");
  std::vector<double> w(2 * (size_t)net->n.nw);
  MGM_HIP(hipMemcpyAsync(w.data(), net->n.w64, sizeof(double2) * net->n.nw, hipMemcpyDeviceToHost,
                         net->n.ctx->stream));
  net->n.ctx->sync();
  std::FILE* f = std::fopen(path, "wb");
  MGM_CHECK(f != nullptr, MGM_ERR_NUMERIC, std::string("cannot open ") + path + " for writing");
  const int32_t L = net->n.L;
  int32_t width[kNetMaxLayers + 1] = {};
  for (int i = 0; i <= L; i++) width[i] = net->n.width[i];
  const int64_t nw = net->n.nw;
  bool ok = std::fwrite(kNetMagic, 1, 8, f) == 8 && std::fwrite(&L, sizeof L, 1, f) == 1 &&
            std::fwrite(width, sizeof width, 1, f) == 1 && std::fwrite(&nw, sizeof nw, 1, f) == 1 &&
            std::fwrite(w.data(), sizeof(double), w.size(), f) == w.size();
  ok = (std::fclose(f) == 0) && ok;
  MGM_CHECK(ok, MGM_ERR_NUMERIC, std::string("write to ") + path + " failed");
  API_END
}

mgm_status mgm_net_load(mgm_net net, const char* path) {
  API_BEGIN
  API_ON(net)
  MGM_CHECK(net && path, MGM_ERR_INVALID_ARG, "NULL argument");
  std::FILE* f = std::fopen(path, "rb");
  MGM_CHECK(f != nullptr, MGM_ERR_INVALID_ARG, std::string("cannot open ") + path);
  char magic[8];
  int32_t L = 0;
  int32_t width[kNetMaxLayers + 1] = {};
  int64_t nw = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kNetMagic, 8) == 0 &&
            std::fread(&L, sizeof L, 1, f) == 1 && std::fread(width, sizeof width, 1, f) == 1 &&
            std::fread(&nw, sizeof nw, 1, f) == 1;
  if (!ok) {
    std::fclose(f);
    throw Error(MGM_ERR_INVALID_ARG, std::string(path) + " is not a network weight file");
  }
  bool same = L == net->n.L && nw == net->n.nw;
  for (int i = 0; same && i <= L && i <= kNetMaxLayers; i++) same = width[i] == net->n.width[i];
  if (!same) {
    std::fclose(f);
    throw Error(MGM_ERR_SHAPE, std::string(path) + " holds a network of other layers or widths");
  }
  std::vector<double> w(2 * (size_t)nw);
  ok = std::fread(w.data(), sizeof(double), w.size(), f) == w.size();
  std::fclose(f);
  MGM_CHECK(ok, MGM_ERR_INVALID_ARG, std::string(path) + " is truncated");
  net->n.upload_weights(w);
  API_END
}

mgm_status mgm_net_apply(mgm_net net, const void* r_dev, void* y_dev, int32_t nrhs) {
  API_BEGIN
  API_ON(net)
  MGM_CHECK(net && r_dev && y_dev, MGM_ERR_INVALID_ARG, "NULL argument");
  net->n.apply((const float2*)r_dev, (float2*)y_dev, nrhs);
  API_END
}

mgm_status mgm_net_loss_grad(mgm_net net, const void* r_dev, const void* e_dev, int32_t nrhs, double* loss,
                             double* grad_host) {
  API_BEGIN
  API_ON(net)
  MGM_CHECK(net && r_dev && e_dev, MGM_ERR_INVALID_ARG, "NULL argument");
  const double l = net->n.loss_grad((const float2*)r_dev, (const float2*)e_dev, nrhs);
  if (loss) *loss = l;
  if (grad_host) {
    MGM_HIP(hipMemcpyAsync(grad_host, net->n.g64, sizeof(double2) * net->n.nw, hipMemcpyDeviceToHost,
                           net->n.ctx->stream));
    net->n.ctx->sync();
  }
  API_END
}

mgm_status mgm_net_train(mgm_net net, mgm_hierarchy h, const mgm_train_desc* desc, mgm_train_stats* stats,
                         double* loss_history) {
  API_BEGIN
  API_ON(net)
  MGM_CHECK(net && h && desc, MGM_ERR_INVALID_ARG, "NULL argument");
  net_train(h->h, net->n, *desc, stats, loss_history);
  API_END
}

void mgm_net_destroy(mgm_net net) {
  if (!net) return;
  if (net->n.pinned) (void)hipHostFree(net->n.pinned);
  delete net;
}

}  // extern "C"

namespace mgm {
SolveCfg solve_cfg_of(const mgm_solve_desc* d) { return cfg_of(d); }
}  // namespace mgm
