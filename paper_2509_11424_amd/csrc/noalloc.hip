// Allocation-free form of the reducing fine dslash (mgm_operator_apply_dot):
// the per-block partial sums of its two reductions live in one fixed device
// array of the library instead of a caller workspace, so the call allocates
// nothing.
//
// `scratch` below is a device symbol.  Host code never passes its name to a
// kernel or a copy: mgm_context_create (the library's set-up call, with its
// device current) looks up the array's device address once per device with
// hipGetSymbolAddress, and the entry point uses that address only.  Each GPU
// holds its own copy of the array for the life of the process.
#include <mutex>

#include "lib.h"

namespace {

constexpr size_t kNoAllocScratchBytes = MGM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace mgm {

void noalloc_bind_device(int device) {
  MGM_CHECK(device >= 0 && device < kMaxDevices, MGM_ERR_INVALID_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] != nullptr) return;
  void* p = nullptr;
  MGM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  MGM_CHECK(p != nullptr && ((uintptr_t)p & 255) == 0, MGM_ERR_HIP, "scratch symbol has no aligned device address");
  g_scratch_ptr[device] = p;
}

static void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  void* p = (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
  MGM_CHECK(p != nullptr, MGM_ERR_INVALID_ARG, "no scratch address for this device (context not created)");
  return p;
}

}  // namespace mgm

using namespace mgm;

extern "C" mgm_status mgm_operator_apply_dot_noalloc(mgm_operator op, mgm_prec prec, const void* x, void* y,
                                                     int32_t nrhs, void* yx_dev, void* yy_dev) {
  try {
    MGM_CHECK(op && x && y && yx_dev && yy_dev, MGM_ERR_INVALID_ARG, "NULL argument");
    MGM_CHECK(nrhs >= 1 && nrhs <= 256, MGM_ERR_INVALID_ARG, "nrhs must be 1..256");
    MGM_CHECK(x != y, MGM_ERR_INVALID_ARG, "x and y must not overlap");
    const int64_t nb = op->op.nblocks(prec, nrhs, true);
    // block partials [2][nrhs][nb], then the segment sums of the finalisation
    const size_t part_entries = (size_t)nb * 2 * nrhs;
    const size_t seg_entries = (size_t)64 * 2 * nrhs;
    // the same count as mgm_operator_dot_workspace_size
    const size_t need_bytes = (part_entries + seg_entries) * sizeof(double2) + 256;
    MGM_CHECK(need_bytes <= kNoAllocScratchBytes, MGM_ERR_WORKSPACE,
              "mgm_operator_apply_dot_noalloc needs " + std::to_string(need_bytes) +
                  " bytes of reduction scratch for this lattice and nrhs; the fixed array holds " +
                  std::to_string(kNoAllocScratchBytes) + " (use mgm_operator_apply_dot with a workspace)");
    DeviceScope on(op->ctx);
    double2* part = (double2*)noalloc_scratch(op->ctx->device);
    Scratch sc;
    sc.partial = part + part_entries;
    sc.cap = seg_entries;
    // every partial the finalisation reads is written by this call's dslash
    // first, so the array needs no clearing between calls
    const int64_t nrun = op->op.apply_dot(prec, x, y, nrhs, part);
    b_finalize_dot_norm(op->ctx, sc, part, nrun, nrhs, (double2*)yx_dev, (double*)yy_dev);
    return MGM_OK;
  } catch (const mgm::Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return MGM_ERR_INVALID_ARG;
  }
}
