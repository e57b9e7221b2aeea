// Block-wide bitonic sort in shared memory with the short compare-exchange
// distances on registers.
#pragma once

#include <hip/hip_runtime.h>

namespace gift {

// Sorts a[0, n) (n a power of two, in shared memory) so that a[i] comes
// before or ties a[i + 1] in the order `before` (a strict weak order: the
// element that comes first), using every thread of the block (blockDim.x a
// multiple of 64).  It is the plain bitonic network: for each merge size k
// and distance j, elements i < i ^ j swap when the upper one comes first
// and (i & k) == 0, or when it does not and (i & k) != 0.  Distances below
// 64 pair lanes of one wave (element i lives in lane i % 64 of its pass),
// so those stages run on registers with `xchg(v, j)` (the value of lane
// lane ^ j) instead of shared memory and a barrier: all merges of up to 64
// elements in one pass, then per merge size k > 64 one barrier per
// distance j >= 64 and one register pass for j < 64.  A pair takes its
// decision from the same two values in both lanes, so ties swap or stay
// together and nothing is duplicated.
template <typename T, typename Before, typename Xchg>
__device__ void block_bitonic_sort(T* a, int n, Before before, Xchg xchg) {
  const int nt = blockDim.x, tid = threadIdx.x;
  auto lds_stage = [&](int k, int j) {
    for (int i = tid; i < n; i += nt) {
      const int ix = i ^ j;
      if (ix > i) {
        const bool up = (i & k) == 0;
        const T x = a[i], y = a[ix];
        if (before(y, x) == up) { a[i] = y; a[ix] = x; }
      }
    }
    __syncthreads();
  };
  if (n < 64) {
    for (int k = 2; k <= n; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) lds_stage(k, j);
    return;
  }
  // one compare-exchange at distance j < 64 on registers (element i)
  auto reg_stage = [&](T v, int i, int k, int j) {
    const T p = xchg(v, j);
    const bool low = (i & j) == 0, up = (i & k) == 0;
    const T& lo = low ? v : p;
    const T& hi = low ? p : v;
    return before(hi, lo) == up ? p : v;
  };
  // n and nt are multiples of 64, so `i < n` holds for whole waves
  for (int i = tid; i < n; i += nt) {
    T v = a[i];
    for (int k = 2; k <= 64; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) v = reg_stage(v, i, k, j);
    a[i] = v;
  }
  __syncthreads();
  for (int k = 128; k <= n; k <<= 1) {
    for (int j = k >> 1; j >= 64; j >>= 1) lds_stage(k, j);
    for (int i = tid; i < n; i += nt) {
      T v = a[i];
      for (int j = 32; j > 0; j >>= 1) v = reg_stage(v, i, k, j);
      a[i] = v;
    }
    __syncthreads();
  }
}

}  // namespace gift
