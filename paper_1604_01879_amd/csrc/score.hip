// Eq. 3 first pass on MFMA: per database shape, the best view similarity
// for every query view, in float32, bfloat16 or e4m3 storage; plus the
// per-view reduced-precision quantizer and the per-query mean.
#include "kernels.h"

namespace gift {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ quantize
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

// One wave per view.
__global__ __launch_bounds__(256) void quantize_kernel(
    const float* __restrict__ src, int64_t n, int dim, int dtype,
    uint8_t* __restrict__ dst, float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  const float* x = src + v * dim;
  float amax = 0.f;
  for (int t = lane; t < dim; t += 64) amax = fmaxf(amax, fabsf(x[t]));
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  const float fmax_ = dtype == GIFT_BF16 ? 1.0f : 448.0f;
  float s = amax / fmax_;
  if (s == 0.f) s = 1.f;
  if (lane == 0) scale[v] = s;
  if (dtype == GIFT_BF16) {
    uint16_t* d = reinterpret_cast<uint16_t*>(dst) + v * dim;
    for (int t = lane; t < dim; t += 64) d[t] = bf16_rne(x[t] / s);
  } else {
    uint8_t* d = dst + v * dim;
    for (int t = lane; t < dim; t += 64) d[t] = e4m3_rne_sat(x[t] / s);
  }
}

void launch_quantize(const float* src, int64_t n, int dim, int dtype,
                     void* dst, float* scale, hipStream_t st) {
  if (n <= 0) return;
  dim3 grid((unsigned)((n + 3) / 4));
  hipLaunchKernelGGL(quantize_kernel, grid, dim3(256), 0, st, src, n, dim,
                     dtype, static_cast<uint8_t*>(dst), scale);
}

// ------------------------------------------------------------------ MFMA tile
// Block tile: BM database rows x BN query views, 4 waves as 2 x 2, each wave
// WM x WN blocks of 32 x 32.  Database rows are laid out 64 per shape (views
// beyond n_views are masked), so a wave's WM*32 rows hold WM/2 whole shapes
// and the per-shape max is taken inside the wave.
//
// K is staged through LDS 128 bytes of each row at a time (32 f32, 64 bf16 or
// 128 e4m3 values).  In a K-tile, lane half h (lanes 32h..32h+31) reads the
// bytes [64h, 64h + 64) of its row as four 16-byte pieces.  The MFMA sums
// over whatever k each (lane half, slot) supplies, and A and B use the same
// assignment, so this permutation of K leaves every dot product unchanged.
constexpr int LROW = 144;  // LDS bytes per staged row: 128 + 16 pad

template <int DT>
struct Mfma;

template <>
struct Mfma<GIFT_F32> {
  // 16 steps of 32x32x2 per K-tile.
  __device__ static __forceinline__ void run(const uint4 (&a)[4], const uint4 (&b)[4], f32x16& c) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a[s].x), __builtin_bit_cast(float, b[s].x), c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a[s].y), __builtin_bit_cast(float, b[s].y), c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a[s].z), __builtin_bit_cast(float, b[s].z), c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a[s].w), __builtin_bit_cast(float, b[s].w), c, 0, 0, 0);
    }
  }
  static constexpr int kstep = 2;  // values summed per accumulation step
};

template <>
struct Mfma<GIFT_BF16> {
  // 4 steps of 32x32x16 per K-tile.
  __device__ static __forceinline__ void run(const uint4 (&a)[4], const uint4 (&b)[4], f32x16& c) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[s]), __builtin_bit_cast(bf16x8, b[s]), c, 0, 0, 0);
  }
  static constexpr int kstep = 16;
};

template <>
struct Mfma<GIFT_FP8E4M3> {
  // 2 steps of 32x32x64 (e4m3 x e4m3, unit block scales) per K-tile.
  __device__ static __forceinline__ void run(const uint4 (&a)[4], const uint4 (&b)[4], f32x16& c) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      i32x8 av = {(int)a[2 * s].x, (int)a[2 * s].y, (int)a[2 * s].z, (int)a[2 * s].w,
                  (int)a[2 * s + 1].x, (int)a[2 * s + 1].y, (int)a[2 * s + 1].z, (int)a[2 * s + 1].w};
      i32x8 bv = {(int)b[2 * s].x, (int)b[2 * s].y, (int)b[2 * s].z, (int)b[2 * s].w,
                  (int)b[2 * s + 1].x, (int)b[2 * s + 1].y, (int)b[2 * s + 1].z, (int)b[2 * s + 1].w};
      c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
    }
  }
  static constexpr int kstep = 64;
};

template <int DT, int WM, int WN>
__global__ __launch_bounds__(256, 1) void score_tiles_kernel(
    const uint8_t* __restrict__ db, const float* __restrict__ db_scale,
    int64_t n_shapes, int n_views, int row_bytes,
    const uint8_t* __restrict__ qv, const float* __restrict__ q_scale,
    int64_t total_q, float* __restrict__ mbuf, int64_t ldm,
    int64_t n_row_tiles, int64_t n_col_tiles) {
  constexpr int BM = 2 * WM * 32;
  constexpr int BN = 2 * WN * 32;
  constexpr int ROWS = BM + BN;
  constexpr int LOADS = ROWS * 8 / 256;  // 16-byte pieces per thread per K-tile
  constexpr int SHAPES_PER_BLOCK = BM / 64;
  static_assert(WM % 2 == 0, "a wave must hold whole shapes");
  extern __shared__ __align__(16) uint8_t lds[];

  // Tile order: GROUP consecutive row tiles share each column sweep, so the
  // blocks on one XCD (ids equal mod 8) keep re-using one database tile.
  constexpr int64_t GROUP = 8;
  const int64_t id = blockIdx.x;
  const int64_t per_group = GROUP * n_col_tiles;
  const int64_t g = id / per_group;
  const int64_t rem = id - g * per_group;
  const int64_t rows_in_group = (n_row_tiles - g * GROUP) < GROUP ? (n_row_tiles - g * GROUP) : GROUP;
  const int64_t row_tile = g * GROUP + rem % rows_in_group;
  const int64_t col_tile = rem / rows_in_group;
  if (row_tile >= n_row_tiles || col_tile >= n_col_tiles) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int half = lane >> 5, l32 = lane & 31;
  const int64_t shape0 = row_tile * SHAPES_PER_BLOCK;
  const int64_t col0 = col_tile * BN;

  // Source pointer of each staged row handled by this thread (nullptr = zero).
  const uint8_t* src[LOADS];
  int piece[LOADS];
#pragma unroll
  for (int it = 0; it < LOADS; ++it) {
    const int idx = tid + 256 * it;
    const int r = idx >> 3;
    piece[it] = idx & 7;
    const uint8_t* p = nullptr;
    if (r < BM) {
      const int64_t shp = shape0 + (r >> 6);
      const int v = r & 63;
      if (shp < n_shapes && v < n_views) p = db + (shp * n_views + v) * (int64_t)row_bytes;
    } else {
      const int64_t c = col0 + (r - BM);
      if (c < total_q) p = qv + c * (int64_t)row_bytes;
    }
    src[it] = p;
  }

  f32x16 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const int n_kt = (row_bytes + 127) / 128;
  uint4 pre[LOADS];
  auto gload = [&](int kt) {
#pragma unroll
    for (int it = 0; it < LOADS; ++it) {
      const int off = kt * 128 + piece[it] * 16;
      if (src[it] != nullptr && off < row_bytes)
        pre[it] = *reinterpret_cast<const uint4*>(src[it] + off);
      else
        pre[it] = make_uint4(0, 0, 0, 0);
    }
  };
  gload(0);
  const uint8_t* arow = lds + (wr * WM * 32 + l32) * LROW + half * 64;
  const uint8_t* brow = lds + (BM + wc * WN * 32 + l32) * LROW + half * 64;
  for (int kt = 0; kt < n_kt; ++kt) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < LOADS; ++it) {
      const int idx = tid + 256 * it;
      *reinterpret_cast<uint4*>(lds + (idx >> 3) * LROW + (idx & 7) * 16) = pre[it];
    }
    __syncthreads();
    if (kt + 1 < n_kt) gload(kt + 1);
    uint4 b[WN][4];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int s = 0; s < 4; ++s)
        b[j][s] = *reinterpret_cast<const uint4*>(brow + j * 32 * LROW + s * 16);
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      uint4 a[4];
#pragma unroll
      for (int s = 0; s < 4; ++s)
        a[s] = *reinterpret_cast<const uint4*>(arow + i * 32 * LROW + s * 16);
#pragma unroll
      for (int j = 0; j < WN; ++j) Mfma<DT>::run(a, b[j], acc[i][j]);
    }
  }

  // Epilogue: lane holds column l32 of each 32x32 block and rows
  // 8*(e/4) + 4*half + (e%4) of it.  Max over the shape's valid views,
  // scales applied per pair (row scale before the max, the positive column
  // scale after it), then combine the two lane halves.
#pragma unroll
  for (int s = 0; s < WM / 2; ++s) {
    const int64_t shp = shape0 + wr * (WM / 2) + s;
    const bool shape_ok = shp < n_shapes;
    float rs[2][16];
    if (DT != GIFT_F32) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int v = bi * 32 + 8 * (e >> 2) + 4 * half + (e & 3);
          rs[bi][e] = (shape_ok && v < n_views) ? db_scale[shp * n_views + v] : 0.f;
        }
    }
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      float m = -INFINITY;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int v = bi * 32 + 8 * (e >> 2) + 4 * half + (e & 3);
          float x = acc[2 * s + bi][j][e];
          if (DT != GIFT_F32) x *= rs[bi][e];
          if (v < n_views) m = fmaxf(m, x);
        }
      m = fmaxf(m, __shfl_xor(m, 32, 64));
      const int64_t c = col0 + wc * WN * 32 + j * 32 + l32;
      if (half == 0 && shape_ok && c < total_q) {
        if (DT != GIFT_F32) m *= q_scale[c];
        mbuf[shp * ldm + c] = m;
      }
    }
  }
}

template <int DT, int WM, int WN>
static gift_status launch_tiles(const gift_views* db, const void* qv,
                                const float* qscale, int64_t total_q,
                                float* mbuf, int64_t ldm, hipStream_t st) {
  constexpr int BM = 2 * WM * 32, BN = 2 * WN * 32;
  const int row_bytes = db->dim * elem_bytes(DT);
  const int64_t n_row_tiles = (db->n_shapes + BM / 64 - 1) / (BM / 64);
  const int64_t n_col_tiles = (total_q + BN - 1) / BN;
  const int64_t blocks = n_row_tiles * n_col_tiles;
  GIFT_CHECK(blocks < (int64_t)1 << 31, GIFT_ECAPACITY, "score grid too large");
  const size_t shmem = (size_t)(BM + BN) * LROW;
  auto kern = score_tiles_kernel<DT, WM, WN>;
  static bool attr_set = false;
  if (!attr_set) {
    GIFT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), shmem, st,
                     static_cast<const uint8_t*>(db->data), db->scale,
                     db->n_shapes, db->n_views, row_bytes,
                     static_cast<const uint8_t*>(qv), qscale, total_q, mbuf,
                     ldm, n_row_tiles, n_col_tiles);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

gift_status launch_score_tiles(const gift_views* db, const void* qv,
                               const float* qscale, int64_t total_q,
                               float* mbuf, int64_t ldm, hipStream_t st) {
  if (total_q <= 0 || db->n_shapes <= 0) return GIFT_OK;
  switch (db->dtype) {
    case GIFT_F32: return launch_tiles<GIFT_F32, 2, 2>(db, qv, qscale, total_q, mbuf, ldm, st);
    case GIFT_BF16: return launch_tiles<GIFT_BF16, 4, 2>(db, qv, qscale, total_q, mbuf, ldm, st);
    case GIFT_FP8E4M3: return launch_tiles<GIFT_FP8E4M3, 4, 2>(db, qv, qscale, total_q, mbuf, ldm, st);
  }
  return fail(GIFT_EUNSUPPORTED, "unknown dtype %d", db->dtype);
}

// ------------------------------------------------------------------ mean
// S[b][p] = (sum over the query's views, ascending) / m.  One thread per
// (query, shape); consecutive threads take consecutive shapes.
__global__ __launch_bounds__(256) void reduce_queries_kernel(
    const float* __restrict__ mbuf, int64_t ldm, int64_t n_shapes,
    const int32_t* __restrict__ qoff, float* __restrict__ S) {
  const int b = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n_shapes) return;
  const int lo = qoff[b], hi = qoff[b + 1];
  const float* row = mbuf + p * ldm;
  float acc = 0.f;
  for (int i = lo; i < hi; ++i) acc += row[i];
  S[(int64_t)b * n_shapes + p] = hi > lo ? acc / (float)(hi - lo) : 0.f;
}

void launch_reduce_queries(const float* mbuf, int64_t ldm, int64_t n_shapes,
                           const int32_t* qoff, int n_queries, float* S,
                           hipStream_t st) {
  if (n_shapes <= 0 || n_queries <= 0) return;
  dim3 grid((unsigned)((n_shapes + 255) / 256), (unsigned)n_queries);
  hipLaunchKernelGGL(reduce_queries_kernel, grid, dim3(256), 0, st, mbuf, ldm,
                     n_shapes, qoff, S);
}

}  // namespace gift
