// Column groups of a block of right-hand sides: the FP16 smoother's vectors
// may store their columns in groups, group-major ([nrhs / gs][rows][gs]).
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

namespace mgm {

// Offset of entry (row, r) of a block of nrhs columns whose columns are
// stored in groups of gs; gs = nrhs is the plain row-major (row, rhs) layout.
__device__ __forceinline__ int64_t grouped_index(int64_t row, int r, int nrhs, int gs, int64_t rows) {
  if (gs == nrhs) return row * nrhs + r;
  const int g = r / gs;
  return ((int64_t)g * rows + row) * gs + (r - g * gs);
}

}  // namespace mgm
