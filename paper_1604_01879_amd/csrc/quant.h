// Per-view scaled reduced-precision codes (shared by the standalone
// quantizer and the batch kernel).
#pragma once

#include "common.h"

namespace gift {

__device__ inline uint16_t bf16_rne(float y) {
  uint32_t u = __builtin_bit_cast(uint32_t, y);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// OCP e4m3fn, round to nearest even, saturating at 448.
__device__ inline uint8_t e4m3_rne_sat(float y) {
  uint32_t sgn = (__builtin_bit_cast(uint32_t, y) >> 24) & 0x80u;
  float a = fabsf(y);
  if (!(a < 448.f)) return (uint8_t)(sgn | 0x7eu);
  if (a < 0.015625f) {                 // below 2^-6: step 2^-9
    int q = (int)rintf(a * 512.f);     // exact scaling, ties to even
    return (uint8_t)(sgn | (uint32_t)q);  // q == 8 encodes 2^-6 exactly
  }
  uint32_t u = __builtin_bit_cast(uint32_t, a);
  u += 0x7ffffu + ((u >> 20) & 1u);    // keep 3 mantissa bits, ties to even
  int e = (int)((u >> 23) & 0xffu) - 127;
  uint32_t m = (u >> 20) & 7u;
  return (uint8_t)(sgn | (uint32_t)((e + 7) << 3) | m);
}

// FP4 e2m1 (values 0, 0.5, 1, 1.5, 2, 3, 4, 6), nearest, ties to even,
// saturating; 4-bit code s:e(2):m(1).
__device__ inline uint8_t e2m1_rne_sat(float y) {
  const uint32_t sgn = (__builtin_bit_cast(uint32_t, y) >> 28) & 0x8u;
  const float a = fabsf(y);
  if (!(a < 6.f)) return (uint8_t)(sgn | 0x7u);
  if (a < 1.f) {                       // step 0.5: codes 0, 1 (0.5), 2 (1.0)
    const int q = (int)rintf(a * 2.f);
    return (uint8_t)(sgn | (uint32_t)q);
  }
  uint32_t u = __builtin_bit_cast(uint32_t, a);
  u += 0x1fffffu + ((u >> 22) & 1u);   // keep 1 mantissa bit, ties to even
  const int e = (int)((u >> 23) & 0xffu) - 127;  // 0..2 (6 stays below the cut)
  const uint32_t m = (u >> 22) & 1u;
  return (uint8_t)(sgn | (uint32_t)((e + 1) << 1) | m);
}

// One wave quantizes view v in MX form: each lane takes whole 32-value
// blocks.  Block exponent floor(log2(amax)) - emax, clamped to [-127, 127].
__device__ inline void quantize_view_mx_wave(const float* __restrict__ src, int64_t v, int dim,
                                             int dtype, uint8_t* __restrict__ dst,
                                             uint8_t* __restrict__ e8m0) {
  const int lane = threadIdx.x & 63;
  const int nblk = dim / 32;
  const int emax = dtype == GIFT_MXFP8 ? 8 : 2;
  const float* x = src + v * dim;
  for (int b = lane; b < nblk; b += 64) {
    float amax = 0.f;
    for (int t = 0; t < 32; ++t) amax = fmaxf(amax, fabsf(x[b * 32 + t]));
    int e = -127;
    if (amax > 0.f) {
      int ex;
      (void)frexpf(amax, &ex);           // amax = m * 2^ex, m in [0.5, 1)
      e = ex - 1 - emax;
      e = e < -127 ? -127 : (e > 127 ? 127 : e);
    }
    e8m0[v * nblk + b] = (uint8_t)(e + 127);
    if (dtype == GIFT_MXFP8) {
      for (int t = 0; t < 32; ++t)
        dst[v * dim + b * 32 + t] = e4m3_rne_sat(ldexpf(x[b * 32 + t], -e));
    } else {
      for (int t = 0; t < 32; t += 2) {
        const uint8_t lo = e2m1_rne_sat(ldexpf(x[b * 32 + t], -e));
        const uint8_t hi = e2m1_rne_sat(ldexpf(x[b * 32 + t + 1], -e));
        dst[(v * dim + b * 32 + t) / 2] = (uint8_t)(lo | (hi << 4));
      }
    }
  }
}

// One wave quantizes view v: scale = max|x| / Fmax (1 for an all-zero
// view), code = round(x / scale).  dim is a multiple of 32: lane l takes the
// float4 pieces l, l + 64, ..., eight pieces' loads in flight, in two passes
// (the maximum, then the codes; the second reads the row from L2).
__device__ inline void quantize_view_wave(const float* __restrict__ src, int64_t v, int dim,
                                          int dtype, uint8_t* __restrict__ dst,
                                          float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const float4* x4 = reinterpret_cast<const float4*>(src + v * dim);
  const int n4 = dim >> 2;
  float amax = 0.f;
  for (int u0 = lane; u0 < n4; u0 += 64 * 8) {
    float4 xa[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      xa[k] = u0 + 64 * k < n4 ? x4[u0 + 64 * k] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      amax = fmaxf(fmaxf(amax, fmaxf(fabsf(xa[k].x), fabsf(xa[k].y))),
                   fmaxf(fabsf(xa[k].z), fabsf(xa[k].w)));
  }
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  const float fmax_ = dtype == GIFT_BF16 ? 1.0f : 448.0f;
  float s = amax / fmax_;
  if (s == 0.f) s = 1.f;
  if (lane == 0) scale[v] = s;
  for (int u0 = lane; u0 < n4; u0 += 64 * 8) {
    float4 xa[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      xa[k] = u0 + 64 * k < n4 ? x4[u0 + 64 * k] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int u = u0 + 64 * k;
      if (u >= n4) continue;
      if (dtype == GIFT_BF16) {
        const uint32_t a = bf16_rne(xa[k].x / s) | ((uint32_t)bf16_rne(xa[k].y / s) << 16);
        const uint32_t b = bf16_rne(xa[k].z / s) | ((uint32_t)bf16_rne(xa[k].w / s) << 16);
        reinterpret_cast<uint2*>(dst + (v * dim) * 2)[u] = make_uint2(a, b);
      } else {
        reinterpret_cast<uint32_t*>(dst + v * dim)[u] =
            (uint32_t)e4m3_rne_sat(xa[k].x / s) | ((uint32_t)e4m3_rne_sat(xa[k].y / s) << 8) |
            ((uint32_t)e4m3_rne_sat(xa[k].z / s) << 16) | ((uint32_t)e4m3_rne_sat(xa[k].w / s) << 24);
      }
    }
  }
}

}  // namespace gift
