// Eq. 3 first pass on MFMA: per database shape, the best view similarity
// for every query view, in float32, bfloat16 or e4m3 storage; plus the
// per-view reduced-precision quantizer and the per-query mean.
#include "kernels.h"
#include "mfma_tile.h"
#include <type_traits>
#include "quant.h"

namespace gift {

// ------------------------------------------------------------------ quantize
// One wave per view.
__global__ __launch_bounds__(256) void quantize_kernel(
    const float* __restrict__ src, int64_t n, int dim, int dtype,
    uint8_t* __restrict__ dst, float* __restrict__ scale) {
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  quantize_view_wave(src, v, dim, dtype, dst, scale);
}

__global__ __launch_bounds__(256) void quantize_mx_kernel(
    const float* __restrict__ src, int64_t n, int dim, int dtype,
    uint8_t* __restrict__ dst, uint8_t* __restrict__ e8m0) {
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v >= n) return;
  quantize_view_mx_wave(src, v, dim, dtype, dst, e8m0);
}

void launch_quantize(const float* src, int64_t n, int dim, int dtype,
                     void* dst, void* scale, hipStream_t st) {
  if (n <= 0) return;
  dim3 grid((unsigned)((n + 3) / 4));
  if (is_mx(dtype))
    hipLaunchKernelGGL(quantize_mx_kernel, grid, dim3(256), 0, st, src, n, dim, dtype,
                       static_cast<uint8_t*>(dst), static_cast<uint8_t*>(scale));
  else
    hipLaunchKernelGGL(quantize_kernel, grid, dim3(256), 0, st, src, n, dim,
                       dtype, static_cast<uint8_t*>(dst), static_cast<float*>(scale));
}

// ------------------------------------------------------------------ MFMA tile
// Database rows are laid out 64 per shape (views beyond n_views read zeros
// and are masked), so a wave's WM*32 rows hold WM/2 whole shapes and the
// per-shape max is taken inside the wave: each lane folds its 32 row values,
// then the two lane halves are combined with one shuffle.
// Tile order: GROUP consecutive row tiles share each column sweep.  Blocks
// are dealt to the 8 XCDs round-robin, so with GROUP a multiple of 8 the
// blocks of one XCD keep to GROUP/8 database tiles while they sweep the
// query tiles, and the database tiles stay in that XCD's L2.  Returns false
// past the last tile.
__device__ __forceinline__ bool tile_coords(int64_t id, int64_t GROUP, int64_t n_row_tiles,
                                            int64_t n_col_tiles, int64_t& row_tile,
                                            int64_t& col_tile) {
  const int64_t per_group = GROUP * n_col_tiles;
  const int64_t g = id / per_group;
  const int64_t rem = id - g * per_group;
  const int64_t rows_in_group = (n_row_tiles - g * GROUP) < GROUP ? (n_row_tiles - g * GROUP) : GROUP;
  row_tile = g * GROUP + rem % rows_in_group;
  col_tile = rem / rows_in_group;
  return row_tile < n_row_tiles && col_tile < n_col_tiles;
}

template <int DT, int WM, int WN, bool DMA, int WC = 2, bool K128 = false, int BST = 2>
__global__ __launch_bounds__(128 * WC, 1) void score_tiles_kernel(
    const uint8_t* __restrict__ db, const void* __restrict__ db_scale_v,
    int64_t n_shapes, int n_views, int row_bytes,
    const uint8_t* __restrict__ qv, const void* __restrict__ q_scale_v,
    int64_t total_q, float* __restrict__ mbuf, int64_t ldm,
    int64_t n_row_tiles, int64_t n_col_tiles, int64_t GROUP) {
  constexpr bool MX = DT == GIFT_MXFP8 || DT == GIFT_MXFP4;
  constexpr bool SCALED = DT == GIFT_BF16 || DT == GIFT_FP8E4M3;  // per-view scales
  const float* db_scale = static_cast<const float*>(db_scale_v);
  const float* q_scale = static_cast<const float*>(q_scale_v);
  using T = TileShape<WM, WN>;
  constexpr int BN = 32 * WC * WN;  // query views per block
  constexpr int SHAPES_PER_BLOCK = T::BM / 64;
  static_assert(WM % 2 == 0, "a wave must hold whole shapes");
  static_assert(WC == 2 || DMA, "4-wave-column tiles use the direct-to-LDS loop");
  extern __shared__ __align__(16) uint8_t lds[];

  int64_t row_tile, col_tile;
  if (!tile_coords(blockIdx.x, GROUP, n_row_tiles, n_col_tiles, row_tile, col_tile)) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int half = lane >> 5, l32 = lane & 31;
  const int64_t shape0 = row_tile * SHAPES_PER_BLOCK;
  const int64_t col0 = col_tile * BN;

  f32x16 acc[WM][WN];
  if constexpr (DMA) {
    // staged rows of this lane as offsets from the block's first database
    // row and first query row (both under 2^32: at most 256 rows of 8 KB);
    // pad rows re-read the first row (their results are never used)
    using D = std::conditional_t<K128, Dma2Shape<WM, WN, WC, BST>, DmaShape<WM, WN, WC>>;
    constexpr int RPI = K128 ? 8 : 16;  // rows per 16-byte load of a wave
    const uint8_t* base_a = db + shape0 * n_views * (int64_t)row_bytes;
    const uint8_t* base_b = qv + col0 * (int64_t)row_bytes;
    uint32_t roff[D::NI];
#pragma unroll
    for (int i = 0; i < D::NI; ++i) {
      const int r = wave * D::WROWS + RPI * i + lane / (64 / RPI);
      uint32_t o = 0;
      if (r < T::BM) {
        const int64_t shp = shape0 + (r >> 6);
        const int v = r & 63;
        if (shp < n_shapes && v < n_views) o = (uint32_t)(((r >> 6) * n_views + v) * row_bytes);
      } else {
        const int64_t c = col0 + (r - T::BM);
        if (c < total_q) o = (uint32_t)((r - T::BM) * row_bytes);
      }
      roff[i] = o;
    }
    if constexpr (K128)
      mfma_tile_mainloop_dma128<DT, WM, WN, WC, BST>(lds, base_a, base_b, roff, row_bytes, acc);
    else
      mfma_tile_mainloop_dma<DT, WM, WN, WC>(lds, base_a, base_b, roff, row_bytes, acc);
  } else {
    const uint8_t* src[T::LOADS];
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
      const int r = staged_row(it);
      const uint8_t* p = nullptr;
      if (r < T::BM) {
        const int64_t shp = shape0 + (r >> 6);
        const int v = r & 63;
        if (shp < n_shapes && v < n_views) p = db + (shp * n_views + v) * (int64_t)row_bytes;
      } else {
        const int64_t c = col0 + (r - T::BM);
        if (c < total_q) p = qv + c * (int64_t)row_bytes;
      }
      src[it] = p;
    }
    if constexpr (MX) {
      // E8M0 rows of the row / column this lane supplies in each block
      const int nblk = (DT == GIFT_MXFP4 ? 2 * row_bytes : row_bytes) / 32;
      const uint8_t* de8 = static_cast<const uint8_t*>(db_scale_v);
      const uint8_t* qe8 = static_cast<const uint8_t*>(q_scale_v);
      const uint8_t* sa_row[WM];
      const uint8_t* sb_row[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        const int r = wr * WM * 32 + i * 32 + l32;
        const int64_t shp = shape0 + (r >> 6);
        const int v = r & 63;
        const bool ok = shp < n_shapes && v < n_views;
        sa_row[i] = de8 + (ok ? (shp * n_views + v) * (int64_t)nblk : 0);
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int64_t c = col0 + wc * WN * 32 + j * 32 + l32;
        sb_row[j] = qe8 + (c < total_q ? c * (int64_t)nblk : 0);
      }
      mfma_tile_mainloop_mx<DT == GIFT_MXFP8 ? 0 : 4, WM, WN>(lds, src, row_bytes, sa_row, sb_row,
                                                              acc);
    } else {
      mfma_tile_mainloop<DT, WM, WN>(lds, src, row_bytes, acc);
    }
  }

  // Epilogue: max over the shape's valid views, the row scale applied
  // before the max and the positive column scale after it.
#pragma unroll
  for (int s = 0; s < WM / 2; ++s) {
    const int64_t shp = shape0 + wr * (WM / 2) + s;
    const bool shape_ok = shp < n_shapes;
    float rs[2][16];
    if (SCALED) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int v = acc_row(bi, e);
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
          const int v = acc_row(bi, e);
          float x = acc[2 * s + bi][j][e];
          if (SCALED) x *= rs[bi][e];
          if (v < n_views) m = fmaxf(m, x);
        }
      m = fmaxf(m, __shfl_xor(m, 32, 64));
      const int64_t c = col0 + wc * WN * 32 + j * 32 + l32;
      if (half == 0 && shape_ok && c < total_q) {
        if (SCALED) m *= q_scale[c];
        mbuf[shp * ldm + c] = m;
      }
    }
  }
}

// Persistent form of the 256 x 256, 8-wave, 128-byte sub-tile kernel (tile
// variant 6, BF16 / e4m3 storage): a grid of one block per CU walks the same
// tile order, block b taking tiles b, b + grid, ...; with the grid a multiple
// of 8 a block's tiles stay on its XCD.  While the last sub-tile of a tile is
// multiplied and its epilogue runs, the first sub-tile of the block's next
// tile and that tile's row and column scales are already loading into LDS,
// so neither a block launch nor the first load's latency is paid per tile.
// Sub-tile kt of the block's running sub-tile count k sits in stage k & 1.
// LDS after the two operand stages: two scale buffers of 256 row scales then
// 256 column scales, used by alternate tiles (wave w loads the scales of the
// 64 rows it stages, a row's scale at index w * 64 + lane), then 256 row
// biases, 0 for a shape's real views and -inf for its pad views, so the
// per-shape maximum of fma(dot, scale, bias) skips pad views without
// per-element masks.
template <int DT>
__global__ __launch_bounds__(512, 1) void score_tiles_persistent_kernel(
    const uint8_t* __restrict__ db, const float* __restrict__ db_scale,
    int64_t n_shapes, int n_views, int row_bytes,
    const uint8_t* __restrict__ qv, const float* __restrict__ q_scale,
    int64_t total_q, float* __restrict__ mbuf, int64_t ldm,
    int64_t n_row_tiles, int64_t n_col_tiles, int64_t GROUP) {
  constexpr int WM = 4, WN = 2, WC = 4;
  using D = Dma2Shape<WM, WN, WC, 2>;
  constexpr int BM = D::BM, BN = D::BN;
  static_assert(D::WROWS == 64 && D::A_STAGE == D::B_STAGE && BM == 256 && BN == 256,
                "64 staged rows per wave, 256 x 256 tile");
  extern __shared__ __align__(16) uint8_t lds[];
  // tile indices, shape and column counts fit 31 bits (checked at launch)
  const uint32_t n_tiles = (uint32_t)(n_row_tiles * n_col_tiles);
  const uint32_t grp = (uint32_t)GROUP, ncols = (uint32_t)n_col_tiles, nrows = (uint32_t)n_row_tiles;
  const int n_shp = (int)n_shapes, n_q = (int)total_q;
  uint32_t id = blockIdx.x;
  if (id >= n_tiles) return;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int wr = wave / WC, wc = wave % WC;
  const int half = lane >> 5, l32 = lane & 31;
  const int n_kt = row_bytes / DMA2_KSUB;
  lds_u8* l3 = (lds_u8*)lds;
  const bool a_wave = wave < BM / 64;           // stages database rows, else query rows
  const int srow = (a_wave ? wave : wave - BM / 64) * 64;  // first row in its side
  const uint32_t side_lds =
      (uint32_t)(uintptr_t)(l3 + (a_wave ? 0 : 2 * D::A_STAGE) + srow * DMA2_KSUB);
  const uint32_t scale_lds = (uint32_t)(uintptr_t)(l3 + D::LDS_BYTES + wave * 256);
  const float* sc_all = reinterpret_cast<const float*>(lds + D::LDS_BYTES);
  float* bias = reinterpret_cast<float*>(lds + D::LDS_BYTES + 4096);
  if (threadIdx.x < BM) bias[threadIdx.x] = (int)(threadIdx.x & 63) < n_views ? 0.f : -INFINITY;

  // This lane stages rows rbase + 8 i of its side.  Tile-invariant offsets
  // from the side's first row, chunk swizzle folded in; a pad view reads the
  // tile's first row.  Rows past the last shape or query column (only in the
  // last row or column tile) keep just the swizzle, i.e. read the first row.
  const int rbase = srow + (lane >> 3);
  uint32_t gfull[D::NI];
#pragma unroll
  for (int i = 0; i < D::NI; ++i) {
    const int rs = rbase + 8 * i;
    const uint32_t sw = (uint32_t)(((lane & 7) ^ dma2_swizzle(rs)) * 16);
    uint32_t o = (uint32_t)(rs * row_bytes);
    if (a_wave) o = (rs & 63) < n_views ? (uint32_t)(((rs >> 6) * n_views + (rs & 63)) * row_bytes) : 0u;
    gfull[i] = o + sw;
  }

  // Sources of tile t: the wave's side base g, this lane's row offsets and
  // the scale address of staged row srow + lane (pad rows read the first
  // scale; their results are never used).
  uint64_t g;
  uint32_t goff[D::NI];
  const float* sp;
  int shape0, col0, nshape0 = 0, ncol0 = 0;
  auto prepare = [&](uint32_t t, int& s0, int& c0) {
    // the tile order of tile_coords, in 32 bits
    const uint32_t per_group = grp * ncols;
    const uint32_t gi = t / per_group;
    const uint32_t rem = t - gi * per_group;
    const uint32_t rows_in_group = nrows - gi * grp < grp ? nrows - gi * grp : grp;
    s0 = (int)(gi * grp + rem % rows_in_group) * (BM / 64);
    c0 = (int)(rem / rows_in_group) * BN;
    g = a_wave ? (uint64_t)(uintptr_t)(db + (int64_t)s0 * n_views * row_bytes)
               : (uint64_t)(uintptr_t)(qv + (int64_t)c0 * row_bytes);
    // rows of this side that exist in the tile
    const int lim = a_wave ? min(n_shp - s0, BM / 64) * 64 : min(n_q - c0, BN);
#pragma unroll
    for (int i = 0; i < D::NI; ++i) goff[i] = rbase + 8 * i < lim ? gfull[i] : gfull[i] & (DMA2_KSUB - 1);
    if (a_wave) {
      const int shp = s0 + wave;
      sp = (shp < n_shp && lane < n_views) ? db_scale + (int64_t)shp * n_views + lane : db_scale;
    } else {
      const int c = c0 + srow + lane;
      sp = c < n_q ? q_scale + c : q_scale;
    }
  };
  auto issue_scales = [&](int buf) {
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dword %0, off"
                 :
                 : "v"(sp), "s"(scale_lds + buf * 2048)
                 : "memory", "m0");
  };

  prepare(id, shape0, col0);
  dma128_issue<D::NI>(side_lds, g, goff);
  issue_scales(0);
  int k0 = 0;   // running sub-tile count of this tile's sub-tile 0, mod 2
  int buf = 0;  // scale buffer of this tile
  for (; id < n_tiles; id += gridDim.x) {
    const uint32_t next = id + gridDim.x;
    f32x16 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
    // sub-tile kt (and at kt = 0 the tile's scales) has landed once this
    // wave's loads are done and all waves meet; after the barrier every wave
    // is past sub-tile kt - 1, whose stage the next load refills
    for (int kt = 0; kt < n_kt; ++kt) {
      wait_vm_barrier<0>();
      const int stage = (k0 + kt) & 1;
      if (kt + 1 < n_kt) {
        dma128_issue<D::NI>(side_lds + (stage ^ 1) * D::A_STAGE,
                            g + (uint64_t)((kt + 1) * DMA2_KSUB), goff);
      } else if (next < n_tiles) {
        // the next tile's sub-tile 0 into the stage sub-tile kt - 1 used,
        // its scales into the buffer the previous tile's epilogue read; the
        // empty asm keeps this set-up here instead of hoisted out of the loop
        uint32_t t = next;
        asm volatile("" : "+s"(t));
        prepare(t, nshape0, ncol0);
        dma128_issue<D::NI>(side_lds + (stage ^ 1) * D::A_STAGE, g, goff);
        issue_scales(buf ^ 1);
      }
      dma128_subtile_mfma<DT, WM, WN, WC>(lds + stage * D::A_STAGE,
                                           lds + 2 * D::A_STAGE + stage * D::B_STAGE, acc);
    }

    // Epilogue: as in score_tiles_kernel, with the scales read from LDS and
    // pad views skipped through their -inf bias.
    const float* rsc = sc_all + buf * 512;
    const float* csc = rsc + 256;
#pragma unroll
    for (int s = 0; s < WM / 2; ++s) {
      const int sh = wr * (WM / 2) + s;  // shape within the tile
      float m[WN];
#pragma unroll
      for (int j = 0; j < WN; ++j) m[j] = -INFINITY;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = sh * 64 + bi * 32 + 8 * q + 4 * half;  // rows acc_row(bi, 4 q .. 4 q + 3)
          const float4 sc4 = *reinterpret_cast<const float4*>(rsc + r);
          const float4 b4 = *reinterpret_cast<const float4*>(bias + r);
          const float scl[4] = {sc4.x, sc4.y, sc4.z, sc4.w}, bs[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
          for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int u = 0; u < 4; ++u)
              m[j] = fmaxf(m[j], fmaf(acc[2 * s + bi][j][4 * q + u], scl[u], bs[u]));
        }
      const int shp = shape0 + sh;
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const float mm = fmaxf(m[j], __shfl_xor(m[j], 32, 64));
        const int cl = wc * WN * 32 + j * 32 + l32;
        const int c = col0 + cl;
        if (half == 0 && shp < n_shp && c < n_q) mbuf[(int64_t)shp * ldm + c] = mm * csc[cl];
      }
      // one shape's scales and biases in registers at a time
      __builtin_amdgcn_sched_barrier(0);
    }
    shape0 = nshape0;
    col0 = ncol0;
    k0 = (k0 + n_kt) & 1;
    buf ^= 1;
  }
}

// Tuning knobs: tile variant per storage dtype and the row-tile group of the
// launch order.  Variants (BF16 / e4m3 storage): for 0..3, bit 0 selects
// 256 x 256 (database rows x query views) instead of 256 x 128 and bit 1 the
// pipelined direct-to-LDS main loop, with 4 waves; 4 is the 256 x 256
// direct-to-LDS tile with 8 waves of 128 x 64 (two per SIMD); 5 and 6 are
// 3 and 4 with 128-byte sub-tiles in two stages; 7 is 6 with three stages
// of query rows; 8, the default and the fastest measured, is 6 as a
// persistent kernel.  The direct loops need rows of whole sub-tiles: 5..8
// fall back to 3 (from 5) or 4 for rows of 64-byte sub-tiles, and 2..4 to
// 0, 1, 1 otherwise.  float32 always uses 128 x 128 and MX storage
// 256 x 128.
static int g_tile[5] = {0, 8, 8, 0, 0};
static int64_t g_group[5] = {8, 32, 32, 8, 8};

gift_status set_score_tuning(int dtype, int tile, int group) {
  GIFT_CHECK(dtype >= 0 && dtype <= 4, GIFT_EINVAL, "bad dtype");
  GIFT_CHECK(tile >= 0 && tile <= 8, GIFT_EINVAL, "tile must be in 0..8");
  GIFT_CHECK(tile == 0 || (dtype == GIFT_BF16 || dtype == GIFT_FP8E4M3), GIFT_EUNSUPPORTED,
             "tile variants 1..8 are for BF16 / FP8 storage");
  GIFT_CHECK(group >= 1 && group <= 1024, GIFT_EINVAL, "group must be in 1..1024");
  if (dtype == GIFT_BF16 || dtype == GIFT_FP8E4M3) g_tile[dtype] = tile;
  g_group[dtype] = group;
  return GIFT_OK;
}

void get_score_tuning(int dtype, int* tile, int* group) {
  *tile = g_tile[dtype];
  *group = (int)g_group[dtype];
}

template <int DT, int WM, int WN, bool DMA = false, int WC = 2, bool K128 = false, int BST = 2>
static gift_status launch_tiles(const gift_views* db, const void* qv,
                                const void* qscale, int64_t total_q,
                                float* mbuf, int64_t ldm, hipStream_t st) {
  constexpr int BM = TileShape<WM, WN>::BM, BN = 32 * WC * WN;
  const int row_bytes = (int)row_bytes_of(DT, db->dim);
  const int64_t n_row_tiles = (db->n_shapes + BM / 64 - 1) / (BM / 64);
  const int64_t n_col_tiles = (total_q + BN - 1) / BN;
  const int64_t blocks = n_row_tiles * n_col_tiles;
  GIFT_CHECK(blocks < (int64_t)1 << 31, GIFT_ECAPACITY, "score grid too large");
  const size_t shmem = !DMA ? TileShape<WM, WN>::LDS_BYTES
                       : K128 ? Dma2Shape<WM, WN, WC, BST>::LDS_BYTES
                              : DmaShape<WM, WN, WC>::LDS_BYTES;
  auto kern = score_tiles_kernel<DT, WM, WN, DMA, WC, K128, BST>;
  {
    const gift_status s = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), shmem);
    if (s != GIFT_OK) return s;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(128 * WC), shmem, st,
                     static_cast<const uint8_t*>(db->data), db->scale,
                     db->n_shapes, db->n_views, row_bytes,
                     static_cast<const uint8_t*>(qv), qscale, total_q, mbuf,
                     ldm, n_row_tiles, n_col_tiles, g_group[DT]);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

// One block per CU (the grid a multiple of 8, so a block's tiles stay on its
// XCD), each walking its share of the tiles.
template <int DT>
static gift_status launch_tiles_persistent(const gift_views* db, const void* qv,
                                           const void* qscale, int64_t total_q,
                                           float* mbuf, int64_t ldm, hipStream_t st) {
  using D = Dma2Shape<4, 2, 4, 2>;
  const int row_bytes = (int)row_bytes_of(DT, db->dim);
  const int64_t n_row_tiles = (db->n_shapes + D::BM / 64 - 1) / (D::BM / 64);
  const int64_t n_col_tiles = (total_q + D::BN - 1) / D::BN;
  const int64_t n_tiles = n_row_tiles * n_col_tiles;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      n_cu <= 0)
    return fail(GIFT_EHIP, "cannot query the device");
  GIFT_CHECK(n_tiles + n_cu < (int64_t)1 << 31 && db->n_shapes < (int64_t)1 << 30 &&
                 total_q < (int64_t)1 << 30,
             GIFT_ECAPACITY, "score grid too large");
  int64_t grid = n_cu >= 8 ? n_cu / 8 * 8 : n_cu;
  if (grid > n_tiles) grid = n_tiles;
  // stages, two scale buffers, row biases
  const size_t shmem = D::LDS_BYTES + (2 * 2 * 256 + 256) * sizeof(float);
  auto kern = score_tiles_persistent_kernel<DT>;
  {
    const gift_status s = ensure_dynamic_lds(reinterpret_cast<const void*>(kern), shmem);
    if (s != GIFT_OK) return s;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(512), shmem, st,
                     static_cast<const uint8_t*>(db->data), static_cast<const float*>(db->scale),
                     db->n_shapes, db->n_views, row_bytes, static_cast<const uint8_t*>(qv),
                     static_cast<const float*>(qscale), total_q, mbuf, ldm, n_row_tiles,
                     n_col_tiles, g_group[DT]);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

gift_status launch_score_tiles(const gift_views* db, const void* qv,
                               const void* qscale, int64_t total_q,
                               float* mbuf, int64_t ldm, hipStream_t st) {
  if (total_q <= 0 || db->n_shapes <= 0) return GIFT_OK;
  switch (db->dtype) {
    case GIFT_F32: return launch_tiles<GIFT_F32, 2, 2>(db, qv, qscale, total_q, mbuf, ldm, st);
    case GIFT_BF16:
    case GIFT_FP8E4M3: {
      int t = g_tile[db->dtype];
      const int rb = row_bytes_of(db->dtype, db->dim);
      if (t >= 5 && rb % DMA2_KSUB != 0) t = t == 5 ? 3 : 4;  // 128-byte sub-tiles -> 64-byte ones
      if (rb % DMA_KSUB != 0) t = t == 4 ? 1 : (t & 1);
#define GIFT_TILE_CASES(DTV)                                                                   \
  switch (t) {                                                                                 \
    case 0: return launch_tiles<DTV, 4, 2>(db, qv, qscale, total_q, mbuf, ldm, st);            \
    case 1: return launch_tiles<DTV, 4, 4>(db, qv, qscale, total_q, mbuf, ldm, st);            \
    case 2: return launch_tiles<DTV, 4, 2, true>(db, qv, qscale, total_q, mbuf, ldm, st);      \
    case 3: return launch_tiles<DTV, 4, 4, true>(db, qv, qscale, total_q, mbuf, ldm, st);      \
    case 4: return launch_tiles<DTV, 4, 2, true, 4>(db, qv, qscale, total_q, mbuf, ldm, st);   \
    case 5: return launch_tiles<DTV, 4, 4, true, 2, true>(db, qv, qscale, total_q, mbuf, ldm,  \
                                                          st);                                 \
    case 6: return launch_tiles<DTV, 4, 2, true, 4, true>(db, qv, qscale, total_q, mbuf, ldm,  \
                                                          st);                                 \
    case 7: return launch_tiles<DTV, 4, 2, true, 4, true, 3>(db, qv, qscale, total_q, mbuf,    \
                                                             ldm, st);                         \
    default: return launch_tiles_persistent<DTV>(db, qv, qscale, total_q, mbuf, ldm, st);      \
  }
      if (db->dtype == GIFT_BF16) GIFT_TILE_CASES(GIFT_BF16)
      GIFT_TILE_CASES(GIFT_FP8E4M3)
#undef GIFT_TILE_CASES
    }
    case GIFT_MXFP8:
      return launch_tiles<GIFT_MXFP8, 4, 2>(db, qv, qscale, total_q, mbuf, ldm, st);
    case GIFT_MXFP4:
      return launch_tiles<GIFT_MXFP4, 4, 2>(db, qv, qscale, total_q, mbuf, ldm, st);
  }
  return fail(GIFT_EUNSUPPORTED, "unknown dtype %d", db->dtype);
}

// ------------------------------------------------------------------ mean
// S[b][p] = (sum over the query's views, ascending) / m.  One block per
// (256 shapes, query): the query's columns of the 256 mbuf rows are staged
// through LDS 64 at a time with one wave reading one 256-byte row segment
// (coalesced), then each thread sums its shape's values in view order.  A
// wave keeps 16 row loads in flight; rows past the last shape and columns
// past the query's last view re-read an in-range element, never summed.
__global__ __launch_bounds__(256) void reduce_queries_kernel(
    const float* __restrict__ mbuf, int64_t ldm, int64_t n_shapes,
    const int32_t* __restrict__ qoff, float* __restrict__ S) {
  __shared__ float tile[256 * 65];
  const int b = blockIdx.y;
  const int64_t p0 = (int64_t)blockIdx.x * 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lo = qoff[b], hi = qoff[b + 1];
  float acc = 0.f;
  for (int c0 = lo; c0 < hi; c0 += 64) {
    const int w = hi - c0 < 64 ? hi - c0 : 64;
    const float* src = mbuf + c0 + (lane < w ? lane : w - 1);
    __syncthreads();
#pragma unroll
    for (int r0 = 0; r0 < 256; r0 += 64) {
      float v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int64_t p = p0 + r0 + wave + 4 * u;
        v[u] = src[(p < n_shapes ? p : n_shapes - 1) * ldm];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) tile[(r0 + wave + 4 * u) * 65 + lane] = v[u];
    }
    __syncthreads();
    for (int i = 0; i < w; ++i) acc += tile[tid * 65 + i];
  }
  const int64_t p = p0 + tid;
  if (p < n_shapes) S[(int64_t)b * n_shapes + p] = hi > lo ? acc / (float)(hi - lo) : 0.f;
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
