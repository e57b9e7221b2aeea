// Internal helpers shared by the GIFT HIP kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/gift.h"

namespace gift {

// ---------------------------------------------------------------- errors
// Records a message for gift_last_error() and returns `st`.
gift_status fail(gift_status st, const char* fmt, ...);

#define GIFT_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      return ::gift::fail(GIFT_EHIP, "%s failed: %s (%s:%d)", #call,          \
                          hipGetErrorString(e_), __FILE__, __LINE__);         \
  } while (0)

#define GIFT_CHECK(cond, st, ...)                                             \
  do {                                                                        \
    if (!(cond)) return ::gift::fail((st), __VA_ARGS__);                      \
  } while (0)

// Launch-error check after a kernel launch.
#define GIFT_LAUNCHED() GIFT_HIP(hipGetLastError())

// Allows `kernel` `bytes` of dynamic LDS on the current device (once per
// kernel and device; thread-safe).
gift_status ensure_dynamic_lds(const void* kernel, size_t bytes);

// ---------------------------------------------------------------- workspace
// Carves 256-byte aligned sub-buffers out of one caller-owned workspace.
// With base == nullptr it only measures.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t bytes() const { return (off + 255) & ~size_t(255); }
};

// Bytes of one stored row of `dim` values.
inline int64_t row_bytes_of(int dtype, int64_t dim) {
  switch (dtype) {
    case GIFT_F32: return 4 * dim;
    case GIFT_BF16: return 2 * dim;
    case GIFT_MXFP4: return dim / 2;
    default: return dim;  // e4m3 and MX e4m3
  }
}
inline bool is_mx(int dtype) { return dtype == GIFT_MXFP8 || dtype == GIFT_MXFP4; }
inline int elem_bytes(int dtype) {
  return dtype == GIFT_F32 ? 4 : dtype == GIFT_BF16 ? 2 : 1;
}

// ---------------------------------------------------------------- ordering
// Maps a float to a uint32 whose unsigned order is the float order
// (NaN-free inputs).  Descending scores use the bitwise complement.
__host__ __device__ inline uint32_t float_order(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float order_float(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __builtin_bit_cast(float, u);
}

// ---------------------------------------------------------------- float-float
// Error-free transformations (Knuth's TwoSum, FMA-based TwoProduct) and the
// compensated dot product of Ogita, Rump and Oishi ("Accurate sum and dot
// product", SIAM J. Sci. Comput. 26(6), 2005), kept as an unevaluated pair
// hi + lo.  Contraction is disabled so the compiler keeps every rounding.
// Global-memory pointers.  Loads through them are global (not flat)
// instructions, which the LDS wait counter does not track.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

// The value of `p` in lane 0 as a global pointer held in scalar registers:
// loads through it take the scalar-base + 32-bit vector-offset form.
template <typename T>
__device__ __forceinline__ gptr<T> uniform_gptr(const T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  return reinterpret_cast<gptr<T>>(((uint64_t)hi << 32) | lo);
}

// The 16-byte T at byte offset `off` from `base`.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ T load_at(gptr<uint8_t> base, uint32_t off) {
  static_assert(sizeof(T) == 16, "16-byte loads");
  return __builtin_bit_cast(T, *reinterpret_cast<gptr<u32x4>>(base + off));
}

struct ff {
  float hi, lo;
};

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e) {
#pragma clang fp contract(off)
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}

// Accumulates x*y into the running compensated sum (s, c).
__device__ __forceinline__ void dot2_step(float x, float y, float& s, float& c) {
#pragma clang fp contract(off)
  float p, ep, es;
  two_prod(x, y, p, ep);
  two_sum(s, p, s, es);
  c = c + (ep + es);
}

// (a.hi + a.lo) + (b.hi + b.lo), renormalised.
__device__ __forceinline__ ff ff_add(ff a, ff b) {
#pragma clang fp contract(off)
  float s, e;
  two_sum(a.hi, b.hi, s, e);
  e = e + (a.lo + b.lo);
  ff r;
  r.hi = s + e;
  r.lo = e - (r.hi - s);
  return r;
}

__device__ __forceinline__ ff ff_norm(float s, float c) {
#pragma clang fp contract(off)
  ff r;
  r.hi = s + c;
  r.lo = c - (r.hi - s);
  return r;
}

// a > b on the represented values (both normalised).
__device__ __forceinline__ bool ff_gt(ff a, ff b) {
  return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo);
}

// (a.hi + a.lo) / n for a small positive integer n.
__device__ __forceinline__ ff ff_div_int(ff a, int n) {
#pragma clang fp contract(off)
  float fn = (float)n;
  float q1 = a.hi / fn;
  float p, e;
  two_prod(q1, fn, p, e);
  float r = ((a.hi - p) - e) + a.lo;   // remainder a - q1*n
  float q2 = r / fn;
  return ff_norm(q1, q2);
}

// Wave-wide (64 lanes) reduction of a compensated sum.
__device__ __forceinline__ ff ff_wave_sum(float s, float c) {
  ff v = ff_norm(s, c);
  for (int o = 32; o > 0; o >>= 1) {
    ff w;
    w.hi = __shfl_xor(v.hi, o, 64);
    w.lo = __shfl_xor(v.lo, o, 64);
    v = ff_add(v, w);
  }
  return v;
}

}  // namespace gift
