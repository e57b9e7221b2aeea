// MFMA main loop shared by the scoring, quantizer and list-scan kernels.
//
// A block of 256 threads (4 waves as 2 x 2) computes a BM x BN tile of
// dot products rows . cols over `row_bytes` bytes per row, BM = 64*WM and
// BN = 64*WN, each wave owning WM x WN blocks of 32 x 32.  The caller gives,
// for every 16-byte piece this thread stages, the source row pointer
// (nullptr reads zeros); rows 0..BM-1 are the A side, BM..BM+BN-1 the B side.
//
// K is staged through LDS 128 bytes of each row at a time (32 f32, 64 bf16
// or 128 e4m3 values).  In a K-tile, lane half h reads bytes [64h, 64h + 64)
// of its row as four 16-byte pieces.  The MFMA sums over whatever k each
// (lane half, slot) supplies and A and B use the same assignment, so this
// permutation of K leaves every dot product unchanged.
//
// Output layout (all 32x32 MFMAs): lane l holds column l % 32 of each block
// and rows 8*(e/4) + 4*(l/32) + (e%4) for accumulator element e.
#pragma once

#include "common.h"

namespace gift {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int LROW = 144;  // LDS bytes per staged row: 128 + 16 pad

template <int DT>
struct Mfma;

struct Pair32 {
  uint4 lo, hi;
};

template <>
struct Mfma<GIFT_F32> {
  // 16 steps of 32x32x2 per K-tile, on one accumulation chain: a dot over d
  // values is within gamma(2 d + 4) sum |x y| of the exact one.
  __device__ static __forceinline__ void run(const uint4 (&a)[4], const uint4 (&b)[4], f32x16& c) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a[s].x), __builtin_bit_cast(float, b[s].x), c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a[s].y), __builtin_bit_cast(float, b[s].y), c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a[s].z), __builtin_bit_cast(float, b[s].z), c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a[s].w), __builtin_bit_cast(float, b[s].w), c, 0, 0, 0);
    }
  }
};

// Pseudo storage type for float32 rows whose K-tiles are summed into a
// fresh block that is then added into the running total: a product is
// rounded once and passes through at most 32 additions in its block and
// one per K-tile after it, so a dot over d values is within
// gamma(48 + d / 32 + 2) sum |x y| of the exact one.  The list scan uses it
// (its tighter first-pass bound lets the rescore drop more candidates);
// the exhaustive float32 tile keeps one chain, whose 16 fewer live
// registers per block keep it at 3 waves per SIMD.
constexpr int MFMA_F32_BLOCKED = 17;

template <>
struct Mfma<MFMA_F32_BLOCKED> {
  __device__ static __forceinline__ void run(const uint4 (&a)[4], const uint4 (&b)[4], f32x16& c) {
    f32x16 p = {};
    Mfma<GIFT_F32>::run(a, b, p);
    c += p;
  }
};

template <>
struct Mfma<GIFT_BF16> {
  // 4 steps of 32x32x16 per K-tile.
  __device__ static __forceinline__ void run(const uint4 (&a)[4], const uint4 (&b)[4], f32x16& c) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[s]), __builtin_bit_cast(bf16x8, b[s]), c, 0, 0, 0);
  }
};

template <>
struct Mfma<GIFT_FP8E4M3> {
  // 2 steps of 32x32x64 (e4m3 x e4m3, unit block scales) per K-tile.
  __device__ static __forceinline__ void run(const uint4 (&a)[4], const uint4 (&b)[4], f32x16& c) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const Pair32 ap = {a[2 * s], a[2 * s + 1]}, bp = {b[2 * s], b[2 * s + 1]};
      c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(__builtin_bit_cast(i32x8, ap),
                                                          __builtin_bit_cast(i32x8, bp), c, 0, 0,
                                                          0, 127, 0, 127);
    }
  }
};

template <int WM, int WN>
struct TileShape {
  static constexpr int BM = 2 * WM * 32;
  static constexpr int BN = 2 * WN * 32;
  static constexpr int ROWS = BM + BN;
  static constexpr int LOADS = ROWS * 8 / 256;  // 16-byte pieces per thread per K-tile
  static constexpr size_t LDS_BYTES = (size_t)ROWS * LROW;
};

// Staged row of the piece `it` of this thread.
__device__ __forceinline__ int staged_row(int it) { return (threadIdx.x + 256 * it) >> 3; }

template <int DT, int WM, int WN>
__device__ __forceinline__ void mfma_tile_mainloop(
    uint8_t* lds, const uint8_t* const (&src)[TileShape<WM, WN>::LOADS], int row_bytes,
    f32x16 (&acc)[WM][WN]) {
  using T = TileShape<WM, WN>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int half = lane >> 5, l32 = lane & 31;

#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const int n_kt = (row_bytes + 127) / 128;
  uint4 pre[T::LOADS];
  auto gload = [&](int kt) {
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
      const int off = kt * 128 + ((tid + 256 * it) & 7) * 16;
      if (src[it] != nullptr && off < row_bytes)
        pre[it] = *reinterpret_cast<const uint4*>(src[it] + off);
      else
        pre[it] = make_uint4(0, 0, 0, 0);
    }
  };
  gload(0);
  const uint8_t* arow = lds + (wr * WM * 32 + l32) * LROW + half * 64;
  const uint8_t* brow = lds + (T::BM + wc * WN * 32 + l32) * LROW + half * 64;
  for (int kt = 0; kt < n_kt; ++kt) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
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
  __syncthreads();  // LDS may be reused by the caller's epilogue
}

// x = hi + lo + r with hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in
// float32), |r| <= 2^-16 |x|; four floats at a time, packed two per word.
// Both roundings are the hardware's round-to-nearest-even pair conversion.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

__device__ __forceinline__ void split_bf16x4(uint4 v, uint2& hi, uint2& lo) {
  const float x0 = __builtin_bit_cast(float, v.x), x1 = __builtin_bit_cast(float, v.y);
  const float x2 = __builtin_bit_cast(float, v.z), x3 = __builtin_bit_cast(float, v.w);
  const uint32_t h01 = bf16_pair(x0, x1), h23 = bf16_pair(x2, x3);
  const float r0 = x0 - __builtin_bit_cast(float, h01 << 16);
  const float r1 = x1 - __builtin_bit_cast(float, h01 & 0xffff0000u);
  const float r2 = x2 - __builtin_bit_cast(float, h23 << 16);
  const float r3 = x3 - __builtin_bit_cast(float, h23 & 0xffff0000u);
  hi = make_uint2(h01, h23);
  lo = make_uint2(bf16_pair(r0, r1), bf16_pair(r2, r3));
}

// Narrow tile for small query-view groups: 128 rows x 32 columns, wave w
// owning rows 32w..32w+31 (one 32 x 32 block); staged rows 0..127 are the A
// side, 128..159 the B side, loaded as in mfma_tile_mainloop.
struct NarrowShape {
  static constexpr int BM = 128;
  static constexpr int BN = 32;
  static constexpr int ROWS = BM + BN;
  static constexpr int LOADS = ROWS * 8 / 256;
  static constexpr size_t LDS_BYTES = (size_t)ROWS * LROW;
};

template <int DT>
__device__ __forceinline__ void mfma_tile_mainloop_narrow(
    uint8_t* lds, const uint8_t* const (&src)[NarrowShape::LOADS], int row_bytes, f32x16& acc) {
  using T = NarrowShape;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;
  const int n_kt = (row_bytes + 127) / 128;
  uint4 pre[T::LOADS];
  auto gload = [&](int kt) {
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
      const int off = kt * 128 + ((tid + 256 * it) & 7) * 16;
      if (src[it] != nullptr && off < row_bytes)
        pre[it] = *reinterpret_cast<const uint4*>(src[it] + off);
      else
        pre[it] = make_uint4(0, 0, 0, 0);
    }
  };
  gload(0);
  const uint8_t* arow = lds + (wave * 32 + l32) * LROW + half * 64;
  const uint8_t* brow = lds + (T::BM + l32) * LROW + half * 64;
  for (int kt = 0; kt < n_kt; ++kt) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
      const int idx = tid + 256 * it;
      *reinterpret_cast<uint4*>(lds + (idx >> 3) * LROW + (idx & 7) * 16) = pre[it];
    }
    __syncthreads();
    if (kt + 1 < n_kt) gload(kt + 1);
    uint4 a[4], b[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      b[s2] = *reinterpret_cast<const uint4*>(brow + s2 * 16);
      a[s2] = *reinterpret_cast<const uint4*>(arow + s2 * 16);
    }
    Mfma<DT>::run(a, b, acc);
  }
  __syncthreads();  // LDS may be reused by the caller's epilogue
}

// Same tile with two LDS stages and global loads issued two K-tiles ahead
// (two register sets), so one barrier per K-tile and about two K-tiles of
// MFMA work to hide each load.  Needs 2 * LDS_BYTES of shared memory.
template <int DT, int WM, int WN>
__device__ __forceinline__ void mfma_tile_mainloop_db(
    uint8_t* lds, const uint8_t* const (&src)[TileShape<WM, WN>::LOADS], int row_bytes,
    f32x16 (&acc)[WM][WN]) {
  using T = TileShape<WM, WN>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int half = lane >> 5, l32 = lane & 31;

#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const int n_kt = (row_bytes + 127) / 128;
  uint4 pre0[T::LOADS], pre1[T::LOADS];
  auto gload = [&](uint4 (&pre)[T::LOADS], int kt) {
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
      const int off = kt * 128 + ((tid + 256 * it) & 7) * 16;
      if (src[it] != nullptr && off < row_bytes)
        pre[it] = *reinterpret_cast<const uint4*>(src[it] + off);
      else
        pre[it] = make_uint4(0, 0, 0, 0);
    }
  };
  auto lstore = [&](const uint4 (&pre)[T::LOADS], uint8_t* buf) {
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
      const int idx = tid + 256 * it;
      *reinterpret_cast<uint4*>(buf + (idx >> 3) * LROW + (idx & 7) * 16) = pre[it];
    }
  };
  auto compute = [&](const uint8_t* buf) {
    const uint8_t* arow = buf + (wr * WM * 32 + l32) * LROW + half * 64;
    const uint8_t* brow = buf + (T::BM + wc * WN * 32 + l32) * LROW + half * 64;
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
  };
  uint8_t* buf0 = lds;
  uint8_t* buf1 = lds + T::LDS_BYTES;
  gload(pre0, 0);
  if (n_kt > 1) gload(pre1, 1);
  lstore(pre0, buf0);
  __syncthreads();
  for (int kt = 0; kt < n_kt; kt += 2) {
    // buf0 holds tile kt; pre1 holds tile kt + 1
    if (kt + 2 < n_kt) gload(pre0, kt + 2);
    compute(buf0);
    if (kt + 1 < n_kt) lstore(pre1, buf1);
    __syncthreads();
    if (kt + 1 >= n_kt) break;
    // buf1 holds tile kt + 1; pre0 holds tile kt + 2
    if (kt + 3 < n_kt) gload(pre1, kt + 3);
    compute(buf1);
    if (kt + 2 < n_kt) lstore(pre0, buf0);
    __syncthreads();
  }
}

// Block-scaled (MX) operands, one E8M0 scale byte per lane per MFMA step;
// FMT is the operand-format code of the scaled MFMA (0: e4m3, 4: e2m1).
//   e4m3: a step covers two 32-value blocks X, Y of the row.  The lane of
//     half h supplies X[16h, 16h+16) then Y[16h, 16h+16) and the scale of
//     block h of the pair (its partner lane carries the other one).  Per
//     128-byte K-tile: steps over blocks (0, 1) and (2, 3); lane half h reads
//     the pieces at bytes 16h, 32 + 16h, 64 + 16h, 96 + 16h.
//   e2m1: a lane supplies one whole 32-value block (16 bytes) with its own
//     scale; half h covers bytes [64h, 64h + 64) in 4 steps.
// `sa`/`sb` hold the lane's scale bytes for the tile's steps, step s in
// byte s.
template <int FMT>
struct MfmaMx;

template <>
struct MfmaMx<0> {
  static constexpr int STEPS = 2;
  // byte offset of the lane half's first piece and the stride between pieces
  __device__ static __forceinline__ int piece0(int half) { return 16 * half; }
  static constexpr int PIECE_STRIDE = 32;
  // scale byte of step s for this lane half: block 2s + half of the K-tile
  __device__ static __forceinline__ uint32_t scales(const uint8_t* row, int kt, int half) {
    const uint8_t* p = row + kt * 4 + half;
    return (uint32_t)p[0] | ((uint32_t)p[2] << 8);
  }
  __device__ static __forceinline__ void run(const uint4 (&a)[4], const uint4 (&b)[4], uint32_t sa,
                                             uint32_t sb, f32x16& c) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const Pair32 ap = {a[2 * s], a[2 * s + 1]}, bp = {b[2 * s], b[2 * s + 1]};
      c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
          __builtin_bit_cast(i32x8, ap), __builtin_bit_cast(i32x8, bp), c, 0, 0, 0,
          (int)((sa >> (8 * s)) & 0xffu), 0, (int)((sb >> (8 * s)) & 0xffu));
    }
  }
};

template <>
struct MfmaMx<4> {
  static constexpr int STEPS = 4;
  __device__ static __forceinline__ int piece0(int half) { return 64 * half; }
  static constexpr int PIECE_STRIDE = 16;
  // scale byte of step s for this lane half: block 4 half + s of the K-tile
  __device__ static __forceinline__ uint32_t scales(const uint8_t* row, int kt, int half) {
    return *reinterpret_cast<const uint32_t*>(row + kt * 8 + half * 4);
  }
  __device__ static __forceinline__ void run(const uint4 (&a)[4], const uint4 (&b)[4], uint32_t sa,
                                             uint32_t sb, f32x16& c) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const Pair32 ap = {a[s], make_uint4(0, 0, 0, 0)}, bp = {b[s], make_uint4(0, 0, 0, 0)};
      c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
          __builtin_bit_cast(i32x8, ap), __builtin_bit_cast(i32x8, bp), c, 4, 4, 0,
          (int)((sa >> (8 * s)) & 0xffu), 0, (int)((sb >> (8 * s)) & 0xffu));
    }
  }
};

// The tile of mfma_tile_mainloop for MX operands.  sa_row[i] / sb_row[j]
// point at the E8M0 bytes of the row / column this lane supplies in block
// i / j (row_bytes must be a multiple of 128).
template <int FMT, int WM, int WN>
__device__ __forceinline__ void mfma_tile_mainloop_mx(
    uint8_t* lds, const uint8_t* const (&src)[TileShape<WM, WN>::LOADS], int row_bytes,
    const uint8_t* const (&sa_row)[WM], const uint8_t* const (&sb_row)[WN],
    f32x16 (&acc)[WM][WN]) {
  using T = TileShape<WM, WN>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int half = lane >> 5, l32 = lane & 31;

#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const int n_kt = row_bytes / 128;
  uint4 pre[T::LOADS];
  auto gload = [&](int kt) {
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
      const int off = kt * 128 + ((tid + 256 * it) & 7) * 16;
      pre[it] = src[it] != nullptr ? *reinterpret_cast<const uint4*>(src[it] + off)
                                   : make_uint4(0, 0, 0, 0);
    }
  };
  auto sload = [&](const uint8_t* row, int kt) -> uint32_t {
    return MfmaMx<FMT>::scales(row, kt, half);
  };
  gload(0);
  constexpr int PS = MfmaMx<FMT>::PIECE_STRIDE;
  const uint8_t* arow = lds + (wr * WM * 32 + l32) * LROW + MfmaMx<FMT>::piece0(half);
  const uint8_t* brow = lds + (T::BM + wc * WN * 32 + l32) * LROW + MfmaMx<FMT>::piece0(half);
  for (int kt = 0; kt < n_kt; ++kt) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
      const int idx = tid + 256 * it;
      *reinterpret_cast<uint4*>(lds + (idx >> 3) * LROW + (idx & 7) * 16) = pre[it];
    }
    __syncthreads();
    if (kt + 1 < n_kt) gload(kt + 1);
    uint32_t sb[WN];
#pragma unroll
    for (int j = 0; j < WN; ++j) sb[j] = sload(sb_row[j], kt);
    uint4 b[WN][4];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int s = 0; s < 4; ++s)
        b[j][s] = *reinterpret_cast<const uint4*>(brow + j * 32 * LROW + s * PS);
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      const uint32_t sa = sload(sa_row[i], kt);
      uint4 a[4];
#pragma unroll
      for (int s = 0; s < 4; ++s)
        a[s] = *reinterpret_cast<const uint4*>(arow + i * 32 * LROW + s * PS);
#pragma unroll
      for (int j = 0; j < WN; ++j) MfmaMx<FMT>::run(a, b[j], sa, sb[j], acc[i][j]);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- DMA loop
// Same tile for BF16 / e4m3 storage with direct global->LDS loads: K in
// 64-byte sub-tiles, DMA_STAGES LDS stages, loads issued DMA_STAGES - 1
// sub-tiles ahead, one barrier per sub-tile and no register staging.  A
// wave's 16-byte load writes 64 consecutive LDS chunks (lane l at chunk l),
// i.e. 16 rows of 64 bytes; rows are unpadded and the 16-byte chunk c of
// row r holds the row's chunk c ^ ((r >> 1) & 3), so the 8 rows read
// together by a lane group hit 8 different bank groups.  row_bytes must be
// a multiple of 64.  Lane l stages rows wave * WROWS + 16 i + l / 4
// (i < NI); rows below BM are read at base_a + roff[i], the others at
// base_b + roff[i] (a 16-row group never straddles BM, so the base is
// uniform per load).  Pad rows may use any readable offset (0): their
// results are not used.
constexpr int DMA_KSUB = 64;
constexpr int DMA_STAGES = 4;

// 2 x WC waves per block: wave w owns rows (w / WC) * WM * 32 .. + WM * 32
// and columns (w % WC) * WN * 32 .. + WN * 32.
template <int WM, int WN, int WC = 2>
struct DmaShape {
  static constexpr int WAVES = 2 * WC;
  static constexpr int BM = 64 * WM;
  static constexpr int BN = 32 * WC * WN;
  static constexpr int ROWS = BM + BN;
  static constexpr int WROWS = ROWS / WAVES;  // rows staged by each wave
  static constexpr int NI = WROWS / 16;       // 16-byte loads per lane per sub-tile
  static constexpr int STAGE_BYTES = ROWS * DMA_KSUB;
  static constexpr size_t LDS_BYTES = (size_t)DMA_STAGES * STAGE_BYTES;
};

typedef __attribute__((address_space(3))) uint8_t lds_u8;

// s_waitcnt vmcnt(n) for the direct loads (issued from inline asm, so the
// compiler does not count them and the vmcnt allowance keeps later
// sub-tiles' loads in flight), then a fenced block barrier, which also
// tells the compiler that every earlier LDS read has completed.
template <int N>
__device__ __forceinline__ void wait_vm_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
  __syncthreads();
}

template <int DT, int WM, int WN, int WC = 2>
__device__ __forceinline__ void mfma_tile_mainloop_dma(
    uint8_t* lds, const uint8_t* base_a, const uint8_t* base_b,
    const uint32_t (&roff)[DmaShape<WM, WN, WC>::NI], int row_bytes, f32x16 (&acc)[WM][WN]) {
  using T = DmaShape<WM, WN, WC>;
  static_assert(DT == GIFT_BF16 || DT == GIFT_FP8E4M3, "BF16 / e4m3 storage only");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int half = lane >> 5, l32 = lane & 31;

#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const int n_kt = row_bytes / DMA_KSUB;
  lds_u8* l3 = (lds_u8*)lds;
  // per-lane offsets of the global chunks this lane copies (row + chunk)
  uint32_t goff[T::NI];
#pragma unroll
  for (int i = 0; i < T::NI; ++i) {
    const int r = wave * T::WROWS + 16 * i + (lane >> 2);
    goff[i] = roff[i] + (uint32_t)(((lane & 3) ^ ((r >> 1) & 3)) * 16);
  }
  // The loads are issued from inline asm so that the compiler does not
  // treat them as pending LDS writes (it would then wait for every one of
  // them before each LDS read); wait_vm_barrier orders them instead.
  const uint32_t wave_lds = (uint32_t)__builtin_amdgcn_readfirstlane(
      (int)(uint32_t)(uintptr_t)(l3 + wave * T::WROWS * DMA_KSUB));
  auto issue = [&](int kt) {
    const uint32_t base = wave_lds + (uint32_t)((kt % DMA_STAGES) * T::STAGE_BYTES);
    const uint8_t* ga = base_a + kt * DMA_KSUB;
    const uint8_t* gb = base_b + kt * DMA_KSUB;
#pragma unroll
    for (int i = 0; i < T::NI; ++i) {
      const bool a_side = wave * T::WROWS + 16 * i < T::BM;  // uniform in the wave
      const uint64_t gv = (uint64_t)(uintptr_t)(a_side ? ga : gb);
      const uint64_t g = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(gv >> 32)) << 32) |
                         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)gv);
      asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1"
                   :
                   : "v"(goff[i]), "s"(g), "s"(base + (uint32_t)(i * 16 * DMA_KSUB))
                   : "memory", "m0");
    }
  };
#pragma unroll
  for (int st = 0; st < DMA_STAGES - 1; ++st)
    if (st < n_kt) issue(st);

  // operand rows all have l32 as their low 5 bits, so one swizzle serves all
  const int sw = (l32 >> 1) & 3;
  const int arow = (wr * WM * 32 + l32) * DMA_KSUB;
  const int brow = (T::BM + wc * WN * 32 + l32) * DMA_KSUB;
  // Logical 16-byte chunk of step s2 that lane half h supplies: BF16 takes
  // chunk 2 s2 + h per 32x32x16 step; e4m3 takes chunks 2h, 2h + 1 (one
  // 32x32x64 step, held as the pair [0], [1]).
  auto chunk = [&](int s2) {
    return DT == GIFT_BF16 ? ((2 * s2 + half) ^ sw) * 16 : ((2 * half + s2) ^ sw) * 16;
  };
  // The B fragments of sub-tile kt + 1 are read from LDS while the MFMAs of
  // sub-tile kt run (two register sets); A fragments are read from the
  // current stage inside the MFMA sequence (that stage is refilled only
  // after the next barrier).
  uint4 fb[WM * WN < 16 ? 2 : 1][WN][2];
  auto read_b = [&](int kt, int set) {
    const uint8_t* st = lds + (kt % DMA_STAGES) * T::STAGE_BYTES;
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
        fb[set][j][s2] = *reinterpret_cast<const uint4*>(st + brow + j * 32 * DMA_KSUB + chunk(s2));
  };
  auto mfmas = [&](int kt, int set) {
    const uint8_t* st = lds + (kt % DMA_STAGES) * T::STAGE_BYTES;
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      uint4 fa[2];
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
        fa[s2] = *reinterpret_cast<const uint4*>(st + arow + i * 32 * DMA_KSUB + chunk(s2));
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        if constexpr (DT == GIFT_BF16) {
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, fa[s2]), __builtin_bit_cast(bf16x8, fb[set][j][s2]),
                acc[i][j], 0, 0, 0);
        } else {
          const Pair32 a = {fa[0], fa[1]}, b = {fb[set][j][0], fb[set][j][1]};
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              __builtin_bit_cast(i32x8, a), __builtin_bit_cast(i32x8, b), acc[i][j], 0, 0, 0, 127,
              0, 127);
        }
      }
    }
  };
  // With 256 accumulator registers (WM x WN = 16) there is no room for a
  // second B set: each sub-tile then waits for its own stage and reads its
  // B fragments itself.
  constexpr bool PREFETCH = WM * WN < 16;
  if constexpr (!PREFETCH) {
    for (int kt = 0; kt < n_kt; ++kt) {
      if (kt + DMA_STAGES - 2 < n_kt) wait_vm_barrier<T::NI * (DMA_STAGES - 2)>();
      else wait_vm_barrier<0>();
      // every wave is past sub-tile kt - 1, so its stage can be refilled
      if (kt + DMA_STAGES - 1 < n_kt) issue(kt + DMA_STAGES - 1);
      read_b(kt, 0);
      mfmas(kt, 0);
    }
  } else {
    // Sub-tile kt is waited for at iteration kt - 1 (kt = 0 before the
    // loop); at that point the loads of at most one later sub-tile are in
    // flight.  Iteration kt then refills the stage of sub-tile kt - 1, whose
    // fragments every wave finished reading before the barrier.
    if (DMA_STAGES - 2 < n_kt) wait_vm_barrier<T::NI * (DMA_STAGES - 2)>();
    else wait_vm_barrier<0>();
    read_b(0, 0);
    // one sub-tile k (k + 1 < n_kt): B fragments of k are in register set
    // `cur`; those of k + 1 go to the other set
    auto step_prefetch = [&](int k, int cur) {
      if (k + DMA_STAGES - 2 < n_kt) wait_vm_barrier<T::NI * (DMA_STAGES - 3)>();
      else wait_vm_barrier<0>();
      if (k + DMA_STAGES - 1 < n_kt) issue(k + DMA_STAGES - 1);
      read_b(k + 1, 1 - cur);
      mfmas(k, cur);
    };
    // The loop body always prefetches, so no path into its MFMAs leaves the
    // current fragments' reads outstanding; the last one or two sub-tiles
    // follow.  (No early exit inside the body: the accumulators stay put.)
    int kt = 0;
    for (; kt + 2 < n_kt; kt += 2) {
      step_prefetch(kt, 0);
      step_prefetch(kt + 1, 1);
    }
    if (kt + 1 < n_kt) {
      step_prefetch(kt, 0);
      mfmas(kt + 1, 1);
    } else {
      mfmas(kt, 0);
    }
  }
  wait_vm_barrier<0>();  // LDS may be reused by the caller
}

// ---------------------------------------------------------- DMA loop, K128
// The same direct global->LDS tile with 128-byte sub-tiles (a whole L2 line
// of each row per sub-tile, so each line is requested once instead of once
// per 64-byte half) and two LDS stages: sub-tile kt + 1 is loaded while the
// MFMAs of kt run, one barrier per 128 bytes of K.  A wave's 16-byte load
// writes 64 consecutive LDS chunks, i.e. 8 rows of 128 bytes; chunk slot s
// of row r holds the row's chunk s ^ dma2_swizzle(r), so any 8 or 16
// consecutive rows read at one logical chunk fall in distinct 16-byte bank
// groups.  row_bytes must be a multiple of 128.  Lane l stages rows
// wave * WROWS + 8 i + l / 8 (i < NI), at base_a + roff[i] below BM and
// base_b + roff[i] above (an 8-row group never straddles BM).
constexpr int DMA2_KSUB = 128;

__device__ __forceinline__ int dma2_swizzle(int r) { return (r & 7) ^ ((r >> 3) & 3); }

// BST: LDS stages of the B side (query rows); the A side always has two.
// With BST = 3 the B rows, which stream through L2 (all query tiles per
// database tile group) and so miss it more often, are loaded two sub-tiles
// ahead.  The A stages come first in LDS, then the B stages.
template <int WM, int WN, int WC = 2, int BST = 2>
struct Dma2Shape {
  static constexpr int WAVES = 2 * WC;
  static constexpr int BM = 64 * WM;
  static constexpr int BN = 32 * WC * WN;
  static constexpr int ROWS = BM + BN;
  static constexpr int WROWS = ROWS / WAVES;  // rows staged by each wave
  static constexpr int NI = WROWS / 8;        // 16-byte loads per lane per sub-tile
  static constexpr int A_STAGE = BM * DMA2_KSUB;
  static constexpr int B_STAGE = BN * DMA2_KSUB;
  static constexpr size_t LDS_BYTES = 2 * (size_t)A_STAGE + (size_t)BST * B_STAGE;
};

// Direct-to-LDS load of one 128-byte sub-tile of a wave's rows: NI 16-byte
// loads per lane, load i reading g + goff[i] and writing the 8 LDS rows
// that start at byte base + 1024 i.  base and g are wave-uniform values the
// compiler cannot always prove uniform (they depend on the wave's side), so
// they are taken from lane 0 into scalar registers.
template <int NI>
__device__ __forceinline__ void dma128_issue(uint32_t base, uint64_t g, const uint32_t (&goff)[NI]) {
  const uint32_t b = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
  const uint64_t gu = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(g >> 32)) << 32) |
                      (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)g);
#pragma unroll
  for (int i = 0; i < NI; ++i)
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1"
                 :
                 : "v"(goff[i]), "s"(gu), "s"(b + (uint32_t)(i * 8 * DMA2_KSUB))
                 : "memory", "m0");
}

// Pseudo storage type of the K128 loop for float32 rows split once into
// BF16 parts (split_bf16x4: x = hi + lo + r, |r| <= 2^-16 |x|): each
// 128-byte sub-tile holds 32 values as 32 high parts then 32 low parts.
// The dot is taken as hi.hi' + hi.lo' + lo.hi' on BF16 MFMA, and each
// sub-tile's 6 MFMAs per 32 x 32 block go into a fresh part added into the
// running total, which bounds the float32 accumulation depth: the result is
// within (3.02 * 2^-16 + 1.02 gamma(6 * 17 + sub-tiles + 2)) sum |x y| of
// the exact dot.
constexpr int DMA_SPLIT_BF16 = 16;

// MFMAs of one staged 128-byte sub-tile: the wave multiplies its WM x WN
// blocks of 32 x 32 (rows wr * WM * 32 + 32 i, columns wc * WN * 32 + 32 j of
// the A stage sta and the B stage stb).  Operand rows all have l32 as their
// low 5 bits, so one swizzle serves all.  BF16 takes logical chunk 2 s + h
// at 32x32x16 step s; e4m3 takes chunks 4 s + 2 h and 4 s + 2 h + 1 at
// 32x32x64 step s.
template <int DT, int WM, int WN, int WC>
__device__ __forceinline__ void dma128_subtile_mfma(const uint8_t* sta, const uint8_t* stb,
                                                    f32x16 (&acc)[WM][WN]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int half = lane >> 5, l32 = lane & 31;
  const int sw = dma2_swizzle(l32);
  const int arow = (wr * WM * 32 + l32) * DMA2_KSUB;
  const int brow = (wc * WN * 32 + l32) * DMA2_KSUB;
  if constexpr (DT == DMA_SPLIT_BF16) {
    // 32 values: chunks 0..3 hold their high parts, 4..7 their low parts;
    // lane half h supplies values 16 h + 8 st .. + 8 at step st.  Per block,
    // hi.hi', hi.lo', lo.hi' of both steps go into a fresh part added into
    // the total (the split loop's products, order and bound).
    uint4 bh[WN][2], bl[WN][2];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        const int c = 2 * half + st;
        bh[j][st] = *reinterpret_cast<const uint4*>(stb + brow + j * 32 * DMA2_KSUB + (c ^ sw) * 16);
        bl[j][st] = *reinterpret_cast<const uint4*>(stb + brow + j * 32 * DMA2_KSUB + ((4 + c) ^ sw) * 16);
      }
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      uint4 ah[2], al[2];
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        const int c = 2 * half + st;
        ah[st] = *reinterpret_cast<const uint4*>(sta + arow + i * 32 * DMA2_KSUB + (c ^ sw) * 16);
        al[st] = *reinterpret_cast<const uint4*>(sta + arow + i * 32 * DMA2_KSUB + ((4 + c) ^ sw) * 16);
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        f32x16 part;
#pragma unroll
        for (int e = 0; e < 16; ++e) part[e] = 0.f;
#pragma unroll
        for (int st = 0; st < 2; ++st) {
          part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[st]),
                                                         __builtin_bit_cast(bf16x8, bh[j][st]), part, 0, 0, 0);
          part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ah[st]),
                                                         __builtin_bit_cast(bf16x8, bl[j][st]), part, 0, 0, 0);
          part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, al[st]),
                                                         __builtin_bit_cast(bf16x8, bh[j][st]), part, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][j][e] += part[e];
      }
    }
    return;
  }
  constexpr int NSTEP = DT == GIFT_BF16 ? 4 : 2;  // MFMA steps per sub-tile
  constexpr int FR = DT == GIFT_BF16 ? 1 : 2;     // 16-byte pieces per lane per step
  auto chunk = [&](int st, int f) {
    return DT == GIFT_BF16 ? ((2 * st + half) ^ sw) * 16 : ((4 * st + 2 * half + f) ^ sw) * 16;
  };
  uint4 fb[WN][NSTEP][FR];
#pragma unroll
  for (int j = 0; j < WN; ++j)
#pragma unroll
    for (int st = 0; st < NSTEP; ++st)
#pragma unroll
      for (int f = 0; f < FR; ++f)
        fb[j][st][f] = *reinterpret_cast<const uint4*>(stb + brow + j * 32 * DMA2_KSUB + chunk(st, f));
#pragma unroll
  for (int i = 0; i < WM; ++i) {
    uint4 fa[NSTEP][FR];
#pragma unroll
    for (int st = 0; st < NSTEP; ++st)
#pragma unroll
      for (int f = 0; f < FR; ++f)
        fa[st][f] = *reinterpret_cast<const uint4*>(sta + arow + i * 32 * DMA2_KSUB + chunk(st, f));
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int st = 0; st < NSTEP; ++st) {
        if constexpr (DT == GIFT_BF16) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8, fa[st][0]), __builtin_bit_cast(bf16x8, fb[j][st][0]),
              acc[i][j], 0, 0, 0);
        } else {
          const Pair32 a = {fa[st][0], fa[st][FR - 1]}, b = {fb[j][st][0], fb[j][st][FR - 1]};
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              __builtin_bit_cast(i32x8, a), __builtin_bit_cast(i32x8, b), acc[i][j], 0, 0, 0,
              127, 0, 127);
        }
      }
  }
}

template <int DT, int WM, int WN, int WC = 2, int BST = 2>
__device__ __forceinline__ void mfma_tile_mainloop_dma128(
    uint8_t* lds, const uint8_t* base_a, const uint8_t* base_b,
    const uint32_t (&roff)[Dma2Shape<WM, WN, WC, BST>::NI], int row_bytes,
    f32x16 (&acc)[WM][WN]) {
  using T = Dma2Shape<WM, WN, WC, BST>;
  static_assert(DT == GIFT_BF16 || DT == GIFT_FP8E4M3 || DT == DMA_SPLIT_BF16,
                "BF16 / e4m3 storage or split float32 rows only");
  static_assert(T::BM % T::WROWS == 0, "a wave stages rows of one side only");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const int n_kt = row_bytes / DMA2_KSUB;
  lds_u8* l3 = (lds_u8*)lds;
  // row r of a side sits at LDS row r of that side's stage; its chunk slot
  // s holds the row's chunk s ^ dma2_swizzle(r)
  uint32_t goff[T::NI];
#pragma unroll
  for (int i = 0; i < T::NI; ++i) {
    const int r = wave * T::WROWS + 8 * i + (lane >> 3);
    const int rs = r < T::BM ? r : r - T::BM;
    goff[i] = roff[i] + (uint32_t)(((lane & 7) ^ dma2_swizzle(rs)) * 16);
  }
  // this wave stages rows of one side: A (database) rows or B (query) rows
  const bool a_wave = wave * T::WROWS < T::BM;  // uniform in the wave
  const int srow = a_wave ? wave * T::WROWS : wave * T::WROWS - T::BM;  // first row in its side
  const uint32_t side_lds = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uintptr_t)(
      l3 + (a_wave ? 0 : 2 * T::A_STAGE) + srow * DMA2_KSUB));
  const uint64_t gv0 = (uint64_t)(uintptr_t)(a_wave ? base_a : base_b);
  const uint64_t gside = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(gv0 >> 32)) << 32) |
                         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)gv0);
  auto issue = [&](int kt) {
    dma128_issue<T::NI>(side_lds + (uint32_t)(a_wave ? (kt & 1) * T::A_STAGE : (kt % BST) * T::B_STAGE),
                        gside + (uint64_t)(kt * DMA2_KSUB), goff);
  };
  // A waves keep one sub-tile in flight, B waves BST - 1
  issue(0);
  if (BST == 3 && !a_wave && 1 < n_kt) issue(1);
  for (int kt = 0; kt < n_kt; ++kt) {
    // this wave's rows of sub-tile kt have landed (a B wave may still have
    // sub-tile kt + 1 in flight); after the barrier every wave is past
    // sub-tile kt - 1, whose stages the next loads refill
    if (BST == 3 && !a_wave && kt + 1 < n_kt) wait_vm_barrier<T::NI>();
    else wait_vm_barrier<0>();
    const int ahead = (BST == 3 && !a_wave) ? 2 : 1;
    if (kt + ahead < n_kt) issue(kt + ahead);
    dma128_subtile_mfma<DT, WM, WN, WC>(lds + (kt & 1) * T::A_STAGE,
                                         lds + 2 * T::A_STAGE + (kt % BST) * T::B_STAGE, acc);
  }
  wait_vm_barrier<0>();  // LDS may be reused by the caller
}

// ------------------------------------------------- narrow tile, DMA loop
// The 128 x 32 narrow tile with direct global->LDS loads of 128-byte
// sub-tiles in NARROW_STAGES stages (two sub-tiles in flight while one is
// multiplied).  Each lane gathers its own rows, so list entries need no
// common base: wave w stages rows 40 w + 8 i + lane / 8 (i < 5) of the 160
// (128 entries, then 32 query views), and chunk slot s of LDS row r holds
// the row's chunk s ^ dma2_swizzle(r).  row_bytes must be a multiple of
// 128, and every src row readable for row_bytes bytes (pad rows point at a
// real row; their results are never used).
constexpr int NARROW_STAGES = 3;
static_assert(NARROW_STAGES >= 2 && NARROW_STAGES <= 4, "the loop waits for up to 2 later sub-tiles");
constexpr int NARROW_NI = NarrowShape::ROWS / 32;  // 16-byte loads per lane per sub-tile
constexpr int NARROW_STAGE_BYTES = NarrowShape::ROWS * DMA2_KSUB;
constexpr size_t NARROW_DMA_LDS_BYTES = (size_t)NARROW_STAGES * NARROW_STAGE_BYTES;

__device__ __forceinline__ int narrow_dma_row(int i) {
  return (int)(threadIdx.x >> 6) * (NarrowShape::ROWS / 4) + 8 * i + (int)((threadIdx.x & 63) >> 3);
}

// The staging pipeline: calls step(stage) once per sub-tile, in order, with
// that sub-tile's 160 rows in LDS (LDS row r at stage + 128 r).
template <typename Step>
__device__ __forceinline__ void narrow_dma_pipeline(uint8_t* lds, const uint8_t* const (&src)[NARROW_NI],
                                                    int row_bytes, Step&& step) {
  static_assert(NarrowShape::ROWS == 4 * 8 * NARROW_NI, "4 waves of 8-row loads");
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n_kt = row_bytes / DMA2_KSUB;
  uint64_t gp[NARROW_NI];
#pragma unroll
  for (int i = 0; i < NARROW_NI; ++i)
    gp[i] = (uint64_t)(uintptr_t)src[i] +
            (uint64_t)(((lane & 7) ^ dma2_swizzle(narrow_dma_row(i))) * 16);
  const uint32_t wave_lds = (uint32_t)__builtin_amdgcn_readfirstlane(
      (int)(uint32_t)(uintptr_t)((lds_u8*)lds + wave * (NarrowShape::ROWS / 4) * DMA2_KSUB));
  auto issue = [&](int kt) {
    const uint32_t base = wave_lds + (uint32_t)((kt % NARROW_STAGES) * NARROW_STAGE_BYTES);
#pragma unroll
    for (int i = 0; i < NARROW_NI; ++i)
      asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off"
                   :
                   : "v"(gp[i] + (uint64_t)(kt * DMA2_KSUB)), "s"(base + (uint32_t)(i * 8 * DMA2_KSUB))
                   : "memory", "m0");
  };
#pragma unroll
  for (int p = 0; p + 1 < NARROW_STAGES; ++p)
    if (p < n_kt) issue(p);
  for (int kt = 0; kt < n_kt; ++kt) {
    // this wave's rows of sub-tile kt have landed (later ones may still be
    // in flight); after the barrier every wave is past sub-tile kt - 1,
    // whose stage the next load refills
    const int later = min(NARROW_STAGES - 2, n_kt - 1 - kt);  // sub-tiles issued after kt
    if (later >= 2) wait_vm_barrier<2 * NARROW_NI>();
    else if (later == 1) wait_vm_barrier<NARROW_NI>();
    else wait_vm_barrier<0>();
    if (kt + NARROW_STAGES - 1 < n_kt) issue(kt + NARROW_STAGES - 1);
    step(lds + (kt % NARROW_STAGES) * NARROW_STAGE_BYTES);
  }
  __syncthreads();  // LDS may be reused by the caller's epilogue
}

// 128 x 32 products: wave w holds rows 32 w .. 32 w + 31 (32x32 accumulator
// layout), with the K-tile MFMAs of Mfma<DT>.
template <int DT>
__device__ __forceinline__ void mfma_tile_mainloop_narrow_dma(
    uint8_t* lds, const uint8_t* const (&src)[NARROW_NI], int row_bytes, f32x16& acc) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5, l32 = lane & 31;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;
  const int sw = dma2_swizzle(l32);
  narrow_dma_pipeline(lds, src, row_bytes, [&](const uint8_t* st) {
    uint4 a[4], b[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int ch = ((4 * half + s2) ^ sw) * 16;
      b[s2] = *reinterpret_cast<const uint4*>(st + (NarrowShape::BM + l32) * DMA2_KSUB + ch);
      a[s2] = *reinterpret_cast<const uint4*>(st + (wave * 32 + l32) * DMA2_KSUB + ch);
    }
    Mfma<DT>::run(a, b, acc);
  });
}

// float32 products of the 128 entries with the first 16 staged query views
// on 16x16x4 MFMA, half the matrix work of the 32-column tile.  Lane l
// supplies row (or column) l % 16 and, in step c of a sub-tile, the value
// at float 8 (l / 16) + c; so lane group g covers floats [8 g, 8 g + 8)
// and the 8 steps together all 32 floats of the sub-tile.  acc[b][t] is
// row 32 w + 16 b + 4 (l / 16) + t, column l % 16.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void mfma_tile_mainloop_narrow16_dma_f32(
    uint8_t* lds, const uint8_t* const (&src)[NARROW_NI], int row_bytes, f32x4 (&acc)[2]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int bk = 0; bk < 2; ++bk)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[bk][t] = 0.f;
  // LDS rows 32 w + 16 b + l16 (entries) and 128 + l16 (query views)
  const int swa0 = dma2_swizzle(l16), swa1 = dma2_swizzle(16 + l16), swb = dma2_swizzle(l16);
  // each sub-tile's 8 MFMAs per block go into a fresh block (as in
  // Mfma<MFMA_F32_BLOCKED>), added into the total during the next sub-tile
  // so the addition does not wait for the MFMA chain before the barrier
  f32x4 prev[2] = {};
  narrow_dma_pipeline(lds, src, row_bytes, [&](const uint8_t* st) {
#pragma unroll
    for (int bk = 0; bk < 2; ++bk) acc[bk] += prev[bk];
    f32x4 part[2] = {};
    uint4 bq[2], aq[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bq[h] = *reinterpret_cast<const uint4*>(st + (NarrowShape::BM + l16) * DMA2_KSUB +
                                              ((2 * g + h) ^ swb) * 16);
      aq[0][h] = *reinterpret_cast<const uint4*>(st + (wave * 32 + l16) * DMA2_KSUB +
                                                 ((2 * g + h) ^ swa0) * 16);
      aq[1][h] = *reinterpret_cast<const uint4*>(st + (wave * 32 + 16 + l16) * DMA2_KSUB +
                                                 ((2 * g + h) ^ swa1) * 16);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const float bv[4] = {__builtin_bit_cast(float, bq[h].x), __builtin_bit_cast(float, bq[h].y),
                           __builtin_bit_cast(float, bq[h].z), __builtin_bit_cast(float, bq[h].w)};
#pragma unroll
      for (int bk = 0; bk < 2; ++bk) {
        const float av[4] = {__builtin_bit_cast(float, aq[bk][h].x), __builtin_bit_cast(float, aq[bk][h].y),
                             __builtin_bit_cast(float, aq[bk][h].z), __builtin_bit_cast(float, aq[bk][h].w)};
#pragma unroll
        for (int c = 0; c < 4; ++c)
          part[bk] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c], bv[c], part[bk], 0, 0, 0);
      }
    }
#pragma unroll
    for (int bk = 0; bk < 2; ++bk) prev[bk] = part[bk];
  });
#pragma unroll
  for (int bk = 0; bk < 2; ++bk) acc[bk] += prev[bk];
}

// Row (within the wave's WM*32 rows) and column of accumulator element e of
// block (i, j) held by this lane.
__device__ __forceinline__ int acc_row(int i, int e) {
  return i * 32 + 8 * (e >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (e & 3);
}
__device__ __forceinline__ int acc_col(int j) { return j * 32 + (threadIdx.x & 31); }

}  // namespace gift
