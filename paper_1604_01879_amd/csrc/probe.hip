// Measurement probe: the sustained matrix-core rate of the 32 x 32 MFMA
// kinds the scorers use, and the shader clock counter beside the constant
// wall clock while it runs.  Not part of the search path.
#include "kernels.h"
#include "mfma_tile.h"

namespace gift {

constexpr int PROBE_CHAINS = 8;  // independent accumulators per wave

template <int DT>
__global__ __launch_bounds__(256) void mfma_probe_kernel(int iters, float* __restrict__ sink,
                                                         unsigned long long* __restrict__ clocks) {
  const int lane = threadIdx.x & 63;
  f32x16 acc[PROBE_CHAINS];
#pragma unroll
  for (int k = 0; k < PROBE_CHAINS; ++k)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[k][e] = e == 0 ? (float)k : 0.f;
  // Mixed-bit operands (the clock under load depends on how many bits
  // toggle), small enough that no accumulator overflows: values below 2^-4
  // (e4m3 bytes 0x08..0x2f), below 1e-3 (BF16, float32).
  auto mix = [&](uint32_t t) {
    uint32_t h = (uint32_t)(lane + 64 * blockIdx.x) * 2654435761u ^ t * 2246822519u;
    h ^= h >> 15;
    h *= 2654435761u;
    return h ^ (h >> 13);
  };
  const float fa = 1e-3f * (float)(mix(1) & 1023) / 1024.f;
  const float fb = 1e-3f * (float)(mix(2) & 1023) / 1024.f;
  bf16x8 ha, hb;
  i32x8 qa, qb;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    ha[t] = (__bf16)(1e-3f * (float)(mix(10 + t) & 1023) / 1024.f);
    hb[t] = (__bf16)(1e-3f * (float)(mix(20 + t) & 1023) / 1024.f);
    uint32_t wa = 0, wb = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wa |= (0x08u + mix(100 + 4 * t + q) % 40u) << (8 * q);
      wb |= (0x08u + mix(200 + 4 * t + q) % 40u) << (8 * q);
    }
    qa[t] = (int)wa;
    qb[t] = (int)wb;
  }
  const unsigned long long c0 = clock64(), w0 = wall_clock64();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) {
      if constexpr (DT == GIFT_F32)
        acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa, fb, acc[k], 0, 0, 0);
      else if constexpr (DT == GIFT_BF16)
        acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha, hb, acc[k], 0, 0, 0);
      else
        acc[k] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(qa, qb, acc[k], 0, 0, 0, 127,
                                                                 0, 127);
    }
  }
  const unsigned long long c1 = clock64(), w1 = wall_clock64();
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < PROBE_CHAINS; ++k)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[k][e];
  sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    clocks[2 * (int64_t)blockIdx.x] = c1 - c0;
    clocks[2 * (int64_t)blockIdx.x + 1] = w1 - w0;
  }
}

}  // namespace gift

using namespace gift;

extern "C" {

gift_status gift_probe_mfma(int32_t dtype, int32_t blocks, int32_t iters, float* sink,
                            uint64_t* clocks, int32_t* wall_khz, void* stream) {
  GIFT_CHECK(dtype == GIFT_F32 || dtype == GIFT_BF16 || dtype == GIFT_FP8E4M3, GIFT_EINVAL,
             "probe dtype must be F32, BF16 or FP8E4M3");
  GIFT_CHECK(blocks >= 1 && iters >= 1 && sink != nullptr && clocks != nullptr &&
                 wall_khz != nullptr,
             GIFT_EINVAL, "bad probe arguments");
  int dev = 0;
  GIFT_HIP(hipGetDevice(&dev));
  GIFT_HIP(hipDeviceGetAttribute(wall_khz, hipDeviceAttributeWallClockRate, dev));
  const hipStream_t st = (hipStream_t)stream;
  auto* ck = reinterpret_cast<unsigned long long*>(clocks);
  switch (dtype) {
    case GIFT_F32:
      hipLaunchKernelGGL(mfma_probe_kernel<GIFT_F32>, dim3(blocks), dim3(256), 0, st, iters, sink, ck);
      break;
    case GIFT_BF16:
      hipLaunchKernelGGL(mfma_probe_kernel<GIFT_BF16>, dim3(blocks), dim3(256), 0, st, iters, sink, ck);
      break;
    default:
      hipLaunchKernelGGL(mfma_probe_kernel<GIFT_FP8E4M3>, dim3(blocks), dim3(256), 0, st, iters, sink, ck);
      break;
  }
  GIFT_LAUNCHED();
  return GIFT_OK;
}

}  // extern "C"
