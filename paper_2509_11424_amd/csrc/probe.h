// Probe generation and time-slice reductions.
#pragma once
#include "common.h"

namespace mgm {

// Z4 entries for probes first .. first+nprobe-1 (see mgm_draw_z4); slice >= 0
// zeroes every site outside time slice `slice` (time-diluted sources).
void draw_z4(Context* c, uint64_t seed, uint32_t stream, uint64_t first, int nprobe, int64_t nsite, int dof,
             mgm_prec prec, void* out, int slice = -1, int64_t sites_per_slice = 1);

// Sites kept by a draw: all, one time slice, and/or one colour of the p^4
// block pattern of a lattice with extents X, Y, Z (probing sources).
struct NoiseMask {
  int slice = -1;
  int64_t sites_per_slice = 1;
  int p = 1;
  int colour = -1;
  int X = 1, Y = 1, Z = 1;
};
// Entries of distribution `kind` (mgm_noise_kind) for probes first .. first+nprobe-1.
void draw_noise(Context* c, int kind, uint64_t seed, uint32_t stream, uint64_t first, int nprobe, int64_t nsite,
                int dof, mgm_prec prec, void* out, const NoiseMask& mk);

constexpr int kMaxSliceVecs = 8;
constexpr int kMaxPairs = 25;
struct SliceArgs {
  const double2* a[kMaxSliceVecs];
  const double2* b[kMaxSliceVecs];
  int ri[kMaxPairs], si[kMaxPairs];
  int npairs;
};
// out[p][rhs][t] (complex), partial: kSliceChunks * npairs * nrhs * T entries
void slice_pairs(Context* c, const SliceArgs& A, int64_t Vs, int T, int nrhs, double2* partial, double2* out);

constexpr int kMaxLoopVecs = 8;
struct LoopArgs {
  const double2* eta;
  const double2* psi[kMaxLoopVecs];
  int nvec;
};
// out[q][gamma][rhs][t]
void loop_gamma(Context* c, const LoopArgs& A, int64_t Vs, int T, int nrhs, double2* partial, double2* out);

constexpr int kSliceChunksHost = 32;

}  // namespace mgm
