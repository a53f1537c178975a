// Shared definitions of the mgmlmc HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <functional>
#include <map>
#include <vector>
#include <stdexcept>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>

#include "../../include/mgmlmc.h"

namespace mgm {

// ------------------------------------------------------------------ errors

struct Error : std::runtime_error {
  mgm_status code;
  Error(mgm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define MGM_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::mgm::Error(MGM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define MGM_CHECK(cond, code, msg)                          \
  do {                                                      \
    if (!(cond)) throw ::mgm::Error((code), (msg));         \
  } while (0)

#define MGM_LAUNCH_CHECK() MGM_HIP(hipGetLastError())

// ----------------------------------------------------------------- complex

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> times_mi(cx<R> a) { return {a.im, -a.re}; }
template <typename R>
__host__ __device__ __forceinline__ R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }
// fused a * b + c (one rounding)
__host__ __device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc += a * b as four fused multiply-adds
template <typename R>
__host__ __device__ __forceinline__ void fma_(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fmar(a.re, b.re, acc.re);
  acc.re = fmar(-a.im, b.im, acc.re);
  acc.im = fmar(a.re, b.im, acc.im);
  acc.im = fmar(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ void fmac_(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fmar(a.re, b.re, acc.re);
  acc.re = fmar(a.im, b.im, acc.re);
  acc.im = fmar(a.re, b.im, acc.im);
  acc.im = fmar(-a.im, b.re, acc.im);
}
// acc += s * a for a real scalar s
template <typename R>
__host__ __device__ __forceinline__ void axpy_(cx<R>& acc, R s, cx<R> a) {
  acc.re = fmar(s, a.re, acc.re);
  acc.im = fmar(s, a.im, acc.im);
}

// -------------------------------------------------------- storage formats

// Storage precision tags: S is the stored complex type, R the arithmetic type.
struct F64 {
  using S = double2;
  using R = double;
  static constexpr mgm_prec prec = MGM_PREC_F64;
  __device__ __forceinline__ static cx<R> ld(const S* p, int64_t i) {
    S v = p[i];
    return {v.x, v.y};
  }
  __device__ __forceinline__ static void st(S* p, int64_t i, cx<R> v) { p[i] = make_double2(v.re, v.im); }
  __device__ __forceinline__ static R ldr(const double* p, int64_t i) { return p[i]; }
  using RS = double;  // stored real type
  // RB consecutive elements starting at i (i a multiple of RB)
  template <int RB>
  __device__ __forceinline__ static void ldv(const S* p, int64_t i, cx<R> (&v)[RB]) {
#pragma unroll
    for (int j = 0; j < RB; j++) v[j] = ld(p, i + j);
  }
  template <int RB>
  __device__ __forceinline__ static void stv(S* p, int64_t i, const cx<R> (&v)[RB]) {
#pragma unroll
    for (int j = 0; j < RB; j++) st(p, i + j, v[j]);
  }
};

struct F32 {
  using S = float2;
  using R = float;
  static constexpr mgm_prec prec = MGM_PREC_F32;
  __device__ __forceinline__ static cx<R> ld(const S* p, int64_t i) {
    S v = p[i];
    return {v.x, v.y};
  }
  __device__ __forceinline__ static void st(S* p, int64_t i, cx<R> v) { p[i] = make_float2(v.re, v.im); }
  using RS = float;
  __device__ __forceinline__ static R ldr(const float* p, int64_t i) { return p[i]; }
  template <int RB>
  __device__ __forceinline__ static void ldv(const S* p, int64_t i, cx<R> (&v)[RB]) {
    if constexpr (RB == 2) {
      const float4 a = *reinterpret_cast<const float4*>(p + i);  // 16-byte aligned: i even
      v[0] = {a.x, a.y};
      v[1] = {a.z, a.w};
    } else {
#pragma unroll
      for (int j = 0; j < RB; j++) v[j] = ld(p, i + j);
    }
  }
  template <int RB>
  __device__ __forceinline__ static void stv(S* p, int64_t i, const cx<R> (&v)[RB]) {
    if constexpr (RB == 2) {
      *reinterpret_cast<float4*>(p + i) = make_float4(v[0].re, v[0].im, v[1].re, v[1].im);
    } else {
#pragma unroll
      for (int j = 0; j < RB; j++) st(p, i + j, v[j]);
    }
  }
};

struct F16 {
  using S = __half2;
  using R = float;
  static constexpr mgm_prec prec = MGM_PREC_F16;
  __device__ __forceinline__ static cx<R> ld(const S* p, int64_t i) {
    float2 v = __half22float2(p[i]);
    return {v.x, v.y};
  }
  __device__ __forceinline__ static void st(S* p, int64_t i, cx<R> v) {
    p[i] = __floats2half2_rn(v.re, v.im);
  }
  using RS = __half;
  __device__ __forceinline__ static R ldr(const __half* p, int64_t i) { return __half2float(p[i]); }
  template <int RB>
  __device__ __forceinline__ static void ldv(const S* p, int64_t i, cx<R> (&v)[RB]) {
    if constexpr (RB == 2) {
      const uint2 a = *reinterpret_cast<const uint2*>(p + i);  // 8-byte aligned: i even
      __half2 h0, h1;
      __builtin_memcpy(&h0, &a.x, 4);
      __builtin_memcpy(&h1, &a.y, 4);
      const float2 f0 = __half22float2(h0), f1 = __half22float2(h1);
      v[0] = {f0.x, f0.y};
      v[1] = {f1.x, f1.y};
    } else {
#pragma unroll
      for (int j = 0; j < RB; j++) v[j] = ld(p, i + j);
    }
  }
  template <int RB>
  __device__ __forceinline__ static void stv(S* p, int64_t i, const cx<R> (&v)[RB]) {
    if constexpr (RB == 2) {
      const __half2 h0 = __floats2half2_rn(v[0].re, v[0].im), h1 = __floats2half2_rn(v[1].re, v[1].im);
      uint2 a;
      __builtin_memcpy(&a.x, &h0, 4);
      __builtin_memcpy(&a.y, &h1, 4);
      *reinterpret_cast<uint2*>(p + i) = a;
    } else {
#pragma unroll
      for (int j = 0; j < RB; j++) st(p, i + j, v[j]);
    }
  }
};

inline size_t prec_bytes(mgm_prec p) {
  switch (p) {
    case MGM_PREC_F64: return 16;
    case MGM_PREC_F32: return 8;
    case MGM_PREC_F16: return 4;
    case MGM_PREC_BF16: return 4;
  }
  return 0;
}

// ------------------------------------------------------------------- arena

// Bump allocator over a caller-owned device workspace.  In sizing mode
// (base == nullptr) it only counts bytes; nothing may be launched then.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  bool sizing() const { return base == nullptr; }
  void* take(size_t bytes) {
    size_t a = (off + 255) & ~size_t(255);
    size_t end = a + ((bytes + 255) & ~size_t(255));
    if (!sizing() && end > cap)
      throw Error(MGM_ERR_WORKSPACE, "workspace too small: need more than " + std::to_string(end) +
                                         " bytes, have " + std::to_string(cap));
    off = end;
    return sizing() ? nullptr : base + a;
  }
  template <typename T>
  T* take_n(size_t n) {
    return reinterpret_cast<T*>(take(n * sizeof(T)));
  }
};

// ---------------------------------------------------------------- context

enum KClass {
  KC_DSLASH_F64 = 0,
  KC_DSLASH_F32 = 1,
  KC_DSLASH_F16 = 2,
  KC_COARSE_F64 = 3,
  KC_COARSE_F32 = 4,
  KC_COARSE_BF16 = 5,
  KC_TRANSFER = 6,
  KC_NET = 7,
  KC_DSLASH_STEP = 8,  // fused FP16 minimal-residual smoother step
  KC_COUNT = 9
};

struct Profiler {
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
    int kclass;
    double bytes;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[KC_COUNT] = {0};
  double ms[KC_COUNT] = {0};
  double bytes[KC_COUNT] = {0};
};

// Launch-shape autotuner: the first call of a kernel for a shape key times
// every variant on the call's own arguments (HIP events, best of three) and
// keeps the fastest; later calls reuse it.  Off by default (variant 0), and
// never active while a stream is being captured into a graph.
struct Tuner {
  bool enabled = false;
  struct Entry {
    int variant = 0;
    std::vector<float> ms;  // timing of every variant
  };
  std::map<std::string, Entry> table;
};

struct Context {
  int device = 0;
  hipStream_t stream = nullptr;
  Profiler prof;
  Tuner tune;
  bool capturing = false;  // stream capture in progress: no timing, no tuning
  // pinned host staging
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  int cu_count = 256;
  size_t max_lds = 65536;  // LDS bytes one workgroup may allocate
  void* host_stage(size_t bytes);
  hipEvent_t take_event();
  void prof_begin(int kclass, double bytes, hipEvent_t* a);
  void prof_end(int kclass, double bytes, hipEvent_t a);
  void prof_flush();
  void sync() { MGM_HIP(hipStreamSynchronize(stream)); }
  // variant of `key` among nvar; run(v) launches variant v on the stream;
  // `dflt` is the variant used while the autotuner is off
  int choose(const std::string& key, int nvar, const std::function<void(int)>& run, int dflt = 0);
};

// RAII timer around one launch of kernel class kc (no-op when profiling is off).
struct ProfScope {
  Context* c;
  int kc;
  double bytes;
  hipEvent_t a = nullptr;
  ProfScope(Context* c_, int kc_, double b_) : c(c_), kc(kc_), bytes(b_) {
    if (c->prof.on && !c->capturing) c->prof_begin(kc, bytes, &a);
  }
  ~ProfScope() {
    if (c->prof.on && a) c->prof_end(kc, bytes, a);
  }
};

// ---------------------------------------------------------- launch helpers

constexpr int kXCD = 8;  // gfx950: 8 accelerator complex dies

// Remaps the hardware workgroup id so that each XCD (which receives
// workgroups round-robin) works on one contiguous range of logical blocks:
// neighbouring lattice sites then share that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t hw, int64_t nblocks) {
  int64_t q = nblocks / kXCD, rem = nblocks % kXCD;
  int64_t x = hw % kXCD, j = hw / kXCD;
  return x * q + (x < rem ? x : rem) + j;
}

inline unsigned nblocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace mgm
