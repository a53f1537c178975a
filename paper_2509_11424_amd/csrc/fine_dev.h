// Device helpers of the Wilson-clover stencil shared by the dslash and the
// Galerkin coarse-operator construction.
#pragma once
#include "fine.h"

namespace mgm {

// Hermitian 6x6 block times a 6-vector, block packed as 6 diagonal reals
// followed by the 15 complex entries below the diagonal.
template <class P>
__device__ __forceinline__ void clover_block(const typename P::RS* __restrict__ C, int64_t V,
                                             int64_t s, int chi, const cx<typename P::R>* x,
                                             cx<typename P::R>* y) {
  using R = typename P::R;
  const typename P::RS* c = C + (int64_t)(36 * chi) * V + s;
#pragma unroll
  for (int i = 0; i < 6; i++) {
    R d = P::ldr(c, (int64_t)i * V);
    y[i] = d * x[i];
  }
  int q = 0;
#pragma unroll
  for (int i = 1; i < 6; i++)
#pragma unroll
    for (int j = 0; j < i; j++, q++) {
      cx<R> cij = {P::ldr(c, (int64_t)(6 + 2 * q) * V), P::ldr(c, (int64_t)(7 + 2 * q) * V)};
      fma_(y[i], cij, x[j]);
      fmac_(y[j], cij, x[i]);
    }
}

// A_mu l (per colour) for the chiral basis, and A_mu^H g.
template <typename R>
__device__ __forceinline__ void A_times(int mu, cx<R> l0, cx<R> l1, cx<R>& o0, cx<R>& o1) {
  switch (mu) {
    case 0: o0 = times_mi(l1); o1 = times_mi(l0); break;        // -i s1
    case 1: o0 = (R)-1 * l1;   o1 = l0; break;                  // -i s2
    case 2: o0 = times_mi(l0); o1 = times_i(l1); break;         // -i s3
    default: o0 = l0; o1 = l1; break;                           // 1
  }
}
template <typename R>
__device__ __forceinline__ void Ad_times(int mu, cx<R> g0, cx<R> g1, cx<R>& o0, cx<R>& o1) {
  switch (mu) {
    case 0: o0 = times_i(g1); o1 = times_i(g0); break;
    case 1: o0 = g1; o1 = (R)-1 * g0; break;
    case 2: o0 = times_i(g0); o1 = times_mi(g1); break;
    default: o0 = g0; o1 = g1; break;
  }
}

}  // namespace mgm
