#include "mg.h"

namespace mgm {

size_t mg_mfma_bytes(const CoarseOp& A) { return 256; }
void mg_mfma_pack(Context*, CoarseOp&) {}
void coarse_apply_mfma(const CoarseOp&, const float2*, float2*, int) {
  throw Error(MGM_ERR_INVALID_ARG, "BF16 MFMA coarse stencil not available");
}

}  // namespace mgm
