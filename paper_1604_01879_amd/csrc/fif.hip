// The first inverted file (Sec. 2.3, Eq. 4, Fig. 2): quantizer c(x) with
// Multiple Assignment, k-means vocabulary, list construction and the list
// scan of a query batch.
#include "kernels.h"
#include "mfma_tile.h"
#include "quant.h"

namespace gift {

// ------------------------------------------------------------------ GEMM
// D[r - r0][k] ~ x_r . b_k in split-BF16 on MFMA, within (3.02 * 2^-16 +
// 1.02 gamma(6 * 17 + dim / 32 + 2)) ||x_r|| ||b_k|| (DMA_SPLIT_BF16), from
// rows split once into BF16 parts (split_bf16x4: hi = bf16(x), lo =
// bf16(x - hi)).  A split row holds, per 32 values, their 32
// high parts (64 bytes) then their 32 low parts, so its 128-byte chunk c is
// sub-tile c of the direct-to-LDS loop (values 32 c .. 32 c + 31).  Rows
// must be a whole number of 32 values.
__global__ __launch_bounds__(256) void split_rows_kernel(const float* __restrict__ src,
                                                         int64_t n_rows, int dim,
                                                         uint8_t* __restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;  // 4 values per thread
  const int per_row = dim / 4;
  if (q >= n_rows * per_row) return;
  const int64_t r = q / per_row;
  const int t = (int)(q - r * per_row) * 4;  // first value
  uint2 hi, lo;
  split_bf16x4(*reinterpret_cast<const uint4*>(src + r * dim + t), hi, lo);
  uint8_t* row = dst + r * (int64_t)dim * 4 + (t / 32) * 128 + (t % 32) * 2;
  *reinterpret_cast<uint2*>(row) = hi;
  *reinterpret_cast<uint2*>(row + 64) = lo;
}

// 256 x 256 tile of D from split rows on the score kernel's direct-to-LDS
// loop (8 waves of 128 x-rows x 64 codewords, two 64 KB stages of 128-byte
// sub-tiles).  Tiles in the score kernel's order, GROUP
// row tiles sharing each column sweep.  xs holds the split rows r0 .. r1 - 1
// (row r at index r - r0).
constexpr int SPLIT_TILE = 256;

//
// With n_rows_dev set, only rows [r0, r0 + *n_rows_dev) (at most r1) are
// computed and blocks past them exit; with `clear` set, the blocks that
// compute also zero words [0, rows * clear_row_words) of `clear` between
// them, stores that drain under the MFMAs.
__global__ __launch_bounds__(512, 1) void dots_split_kernel(
    const uint8_t* __restrict__ xs, int64_t r0, int64_t r1, const uint8_t* __restrict__ cbs, int K,
    int dim, float* __restrict__ D, int64_t n_row_tiles, int64_t n_col_tiles,
    const int32_t* __restrict__ n_rows_dev, uint32_t* __restrict__ clear,
    int64_t clear_row_words) {
  constexpr int WM = 4, WN = 2, WC = 4;
  using S = Dma2Shape<WM, WN, WC, 2>;
  static_assert(S::BM == SPLIT_TILE && S::BN == SPLIT_TILE, "256 x 256 tiles");
  extern __shared__ __align__(16) uint8_t lds[];
  constexpr int64_t GROUP = 8;
  const int64_t id = blockIdx.x;
  const int64_t per_group = GROUP * n_col_tiles;
  const int64_t gi = id / per_group;
  const int64_t rem = id - gi * per_group;
  const int64_t rows_in_group = n_row_tiles - gi * GROUP < GROUP ? n_row_tiles - gi * GROUP : GROUP;
  const int64_t row_tile = gi * GROUP + rem % rows_in_group;
  const int64_t col_tile = rem / rows_in_group;
  if (n_rows_dev != nullptr) {
    const int64_t nr = *n_rows_dev;
    if (r0 + nr < r1) r1 = r0 + (nr > 0 ? nr : 0);
    const int64_t act_rt = (r1 - r0 + SPLIT_TILE - 1) / SPLIT_TILE;
    if (row_tile >= act_rt) return;  // block-uniform
    if (clear != nullptr) {
      const int64_t words = (r1 - r0) * clear_row_words, blocks = act_rt * n_col_tiles;
      const int64_t per = ((words + blocks - 1) / blocks + 2047) / 2048 * 2048;
      const int64_t e0 = (row_tile * n_col_tiles + col_tile) * per;
      const int64_t e1 = e0 + per < words ? e0 + per : words;
      for (int64_t e = e0 + 4 * threadIdx.x; e < e1; e += 2048) {
        if (e + 4 <= e1)
          *reinterpret_cast<uint4*>(clear + e) = make_uint4(0u, 0u, 0u, 0u);
        else
          for (int64_t t = e; t < e1; ++t) clear[t] = 0u;
      }
    }
  }
  const int64_t rb = r0 + row_tile * SPLIT_TILE;  // first x row of the tile
  const int64_t cb0 = col_tile * SPLIT_TILE;      // first codeword
  const int row_bytes = dim * 4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave / WC, wc = wave % WC;
  // staged rows as offsets from the tile's first x row and first codeword
  // (under 2^32: 256 rows of at most 16 MB); pad rows re-read the first
  uint32_t roff[S::NI];
#pragma unroll
  for (int i = 0; i < S::NI; ++i) {
    const int r = wave * S::WROWS + 8 * i + lane / 8;
    uint32_t o = 0;
    if (r < S::BM) {
      if (rb + r < r1) o = (uint32_t)(r * row_bytes);
    } else if (cb0 + (r - S::BM) < K) {
      o = (uint32_t)((r - S::BM) * row_bytes);
    }
    roff[i] = o;
  }
  f32x16 acc[WM][WN];
  mfma_tile_mainloop_dma128<DMA_SPLIT_BF16, WM, WN, WC>(
      lds, xs + (rb - r0) * (int64_t)row_bytes, cbs + cb0 * (int64_t)row_bytes, roff, row_bytes,
      acc);
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t r = rb + wr * WM * 32 + acc_row(i, e);
        const int64_t k = cb0 + wc * WN * 32 + acc_col(j);
        if (r < r1 && k < K) D[(r - r0) * K + k] = acc[i][j][e];
      }
}

void launch_split_rows(const float* src, int64_t n, int dim, uint8_t* dst, hipStream_t st) {
  const int64_t q = n * (dim / 4);
  if (q <= 0) return;
  hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, st, src, n,
                     dim, dst);
}

// One wave splits row v of x into dst (the split_rows_kernel layout).
__device__ __forceinline__ void split_row_wave(const float* __restrict__ x, int64_t v, int dim,
                                               uint8_t* __restrict__ dst) {
  const int lane = threadIdx.x & 63;
  const float* src = x + v * dim;
  uint8_t* row = dst + v * (int64_t)dim * 4;
#pragma unroll 8
  for (int t = lane * 4; t < dim; t += 256) {
    uint2 hi, lo;
    split_bf16x4(*reinterpret_cast<const uint4*>(src + t), hi, lo);
    uint8_t* o = row + (t / 32) * 128 + (t % 32) * 2;
    *reinterpret_cast<uint2*>(o) = hi;
    *reinterpret_cast<uint2*>(o + 64) = lo;
  }
}

// 128 x 128 tile of D (rows of xs, codewords of cbs, both split) for a
// 4-wave block with 64 KB of LDS: the direct-to-LDS loop with 64 x 64 per
// wave.  Same products, order and bound as dots_split_kernel, so the same
// D.
__device__ __forceinline__ void dots_split_tile(const uint8_t* __restrict__ xs, int64_t n_rows,
                                                const uint8_t* __restrict__ cbs, int K, int dim,
                                                float* __restrict__ D, int64_t row_tile,
                                                int64_t col_tile, uint8_t* lds) {
  constexpr int WM = 2, WN = 2, WC = 2;
  using S = Dma2Shape<WM, WN, WC, 2>;
  const int64_t rb = row_tile * S::BM, cb0 = col_tile * S::BN;
  const int row_bytes = dim * 4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave / WC, wc = wave % WC;
  uint32_t roff[S::NI];
#pragma unroll
  for (int i = 0; i < S::NI; ++i) {
    const int r = wave * S::WROWS + 8 * i + lane / 8;
    uint32_t o = 0;
    if (r < S::BM) {
      if (rb + r < n_rows) o = (uint32_t)(r * row_bytes);
    } else if (cb0 + (r - S::BM) < K) {
      o = (uint32_t)((r - S::BM) * row_bytes);
    }
    roff[i] = o;
  }
  f32x16 acc[WM][WN];
  mfma_tile_mainloop_dma128<DMA_SPLIT_BF16, WM, WN, WC>(
      lds, xs + rb * (int64_t)row_bytes, cbs + cb0 * (int64_t)row_bytes, roff, row_bytes, acc);
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t r = rb + wr * WM * 32 + acc_row(i, e);
        const int64_t k = cb0 + wc * WN * 32 + acc_col(j);
        if (r < n_rows && k < K) D[r * K + k] = acc[i][j][e];
      }
}

// ------------------------------------------------------------------ norms
// ||b_k||^2 as a compensated sum, one wave per codeword.
__global__ __launch_bounds__(256) void norms_kernel(const float* __restrict__ cb, int K, int dim,
                                                    float* __restrict__ nhi, float* __restrict__ nlo) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= K) return;
  const float* b = cb + (int64_t)k * dim;
  float s = 0.f, c = 0.f;
  for (int t = lane; t < dim; t += 64) dot2_step(b[t], b[t], s, c);
  const ff v = ff_wave_sum(s, c);
  if (lane == 0) { nhi[k] = v.hi; nlo[k] = v.lo; }
}

// ------------------------------------------------------------------ select
// d^_k = ||b_k||^2 - 2 D[k] in float32 with a per-k bound e_k; U = the
// ma-th smallest d^_k + e_k bounds the true ma-th smallest distance from
// above, so every k with d^_k - e_k <= U may belong to the exact top-ma.
// Those candidates are re-evaluated with compensated arithmetic and the ma
// smallest (distance, index) are written.
constexpr int SEL_CAP = 256;   // candidates kept per row
constexpr int MAX_MA = 8;
constexpr int SEL_UNROLL = 16;  // codewords per lane with loads in flight together

__device__ inline bool dk_less(float ah, float al, int ak, float bh, float bl, int bk) {
  if (ah != bh) return ah < bh;
  if (al != bl) return al < bl;
  return ak < bk;
}

// d^_k and its bound e_k from the float32 dot dv and ||b_k||^2 (hi part) nv.
__device__ __forceinline__ void sel_bounds(float dv, float nv, float c1, float c2, float& dk,
                                           float& ek) {
  dk = nv - 2.f * dv;
  ek = c1 * sqrtf(fmaxf(nv, 0.f)) + c2 * (fabsf(dk) + 1.f);
}

// LDS of a selection item: per wave its candidates (index, lower bound,
// compensated distance) and its ma smallest upper bounds and count, and a
// block-wide candidate list for rows split over the four waves.
struct SelLds {
  int wk[4][SEL_CAP];
  float wlb[4][SEL_CAP];
  float chi[4][SEL_CAP], clo[4][SEL_CAP];
  int cand[SEL_CAP];
  float wub[4][MAX_MA];
  int wn[4];
};
constexpr size_t SEL_LDS = sizeof(SelLds);

// Certified ma nearest codewords of rows of the chunk [r0, r1); D holds the
// chunk's dots.  SPLIT: one row per block (row r0 + blk), wave w scanning the
// codewords [w kq, (w + 1) kq) (kq = K / 4 rounded up to 64), so the passes
// over D are a quarter as long and the candidates' compensated dots run four
// at a time.  Otherwise one row per wave (rows r0 + 4 blk + w; an idle wave
// past the last row redoes it and writes nothing).  With `counts` set
// (ma == 1), the chosen word's counter is incremented.  The word is stored,
// and counted, through device-scope atomics.
template <bool SPLIT>
__device__ __forceinline__ void select_rows(const float* __restrict__ x, int64_t r0, int64_t r1,
                                            const float* __restrict__ cb, int K, int dim, int ma,
                                            const float* __restrict__ D,
                                            const float* __restrict__ nhi,
                                            const float* __restrict__ nlo, float gamma2,
                                            int32_t* __restrict__ words,
                                            int32_t* __restrict__ overflow,
                                            int32_t* __restrict__ counts, int64_t blk,
                                            uint8_t* smem) {
  SelLds& L = *reinterpret_cast<SelLds*>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r_raw = SPLIT ? r0 + blk : r0 + blk * 4 + wave;
  if (SPLIT && r_raw >= r1) return;  // block-uniform
  const bool active = r_raw < r1;
  const int64_t r = active ? r_raw : r1 - 1;
  const float* xr = x + r * dim;
  const float* Dr = D + (r - r0) * K;
  // ||x|| with slack for its own rounding (lane l: float4 pieces l, l + 64,
  // ...; dim is a multiple of 32, so the piece count is a multiple of 8)
  const int n4 = dim >> 2;
  const float4* x4 = reinterpret_cast<const float4*>(xr);
  float ss = 0.f;
  for (int u0 = lane; u0 < n4; u0 += 64 * 8) {
    float4 xa[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      xa[k] = u0 + 64 * k < n4 ? x4[u0 + 64 * k] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      ss = __builtin_fmaf(xa[k].x, xa[k].x, ss);
      ss = __builtin_fmaf(xa[k].y, xa[k].y, ss);
      ss = __builtin_fmaf(xa[k].z, xa[k].z, ss);
      ss = __builtin_fmaf(xa[k].w, xa[k].w, ss);
    }
  }
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
  const float xn = sqrtf(ss) * 1.001f + 1e-30f;
  const float c1 = gamma2 * xn;
  const float c2 = 2.4e-7f;  // a few float32 roundings of d^_k itself
  const int kq = SPLIT ? ((K + 3) / 4 + 63) / 64 * 64 : K;
  const int kb = SPLIT ? min(K, wave * kq) : 0, ke = SPLIT ? min(K, kb + kq) : K;

  // This wave's candidates so far (n_w, the first SEL_CAP kept).
  int n_w = 0;
  bool rescan = true;  // collect this wave's candidates in a second pass
  if (ma == 1) {
    // One pass.  The running U (smallest upper bound so far, over whole
    // blocks of 64 SEL_UNROLL codewords) never falls below the final U, so
    // every final candidate passes the test against it and is kept, in
    // ascending k, with its lower bound; the final U filters them below.
    float Uw = INFINITY;
    for (int k0 = kb; k0 < ke; k0 += 64 * SEL_UNROLL) {
      float dv[SEL_UNROLL], nv[SEL_UNROLL], lb[SEL_UNROLL];
#pragma unroll
      for (int t = 0; t < SEL_UNROLL; ++t) {
        const int k = k0 + 64 * t + lane;
        dv[t] = k < ke ? Dr[k] : 0.f;
        nv[t] = k < ke ? nhi[k] : 0.f;
      }
      float umin = INFINITY;
#pragma unroll
      for (int t = 0; t < SEL_UNROLL; ++t) {
        lb[t] = INFINITY;
        if (k0 + 64 * t + lane < ke) {
          float dk, ek;
          sel_bounds(dv[t], nv[t], c1, c2, dk, ek);
          umin = fminf(umin, dk + ek);
          lb[t] = dk - ek;
        }
      }
      for (int o = 32; o > 0; o >>= 1) umin = fminf(umin, __shfl_xor(umin, o, 64));
      Uw = fminf(Uw, umin);
#pragma unroll
      for (int t = 0; t < SEL_UNROLL; ++t) {
        const bool f = lb[t] <= Uw;
        const unsigned long long bal = __ballot(f);
        const int pos = n_w + __popcll(bal & ((1ull << lane) - 1ull));
        if (f && pos < SEL_CAP) {
          L.wk[wave][pos] = k0 + 64 * t + lane;
          L.wlb[wave][pos] = lb[t];
        }
        n_w += __popcll(bal);
      }
    }
    if (lane == 0) L.wub[wave][0] = Uw;
    rescan = n_w > SEL_CAP;
  } else {
    // lane-local ma smallest upper bounds; SEL_UNROLL codewords per lane are
    // loaded before any is used, so their loads overlap
    float best[MAX_MA];
#pragma unroll
    for (int a = 0; a < MAX_MA; ++a) best[a] = INFINITY;
    for (int k0 = kb + lane; k0 < ke; k0 += 64 * SEL_UNROLL) {
      float dv[SEL_UNROLL], nv[SEL_UNROLL];
#pragma unroll
      for (int t = 0; t < SEL_UNROLL; ++t) {
        const int k = k0 + 64 * t;
        dv[t] = k < ke ? Dr[k] : 0.f;
        nv[t] = k < ke ? nhi[k] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < SEL_UNROLL; ++t) {
        if (k0 + 64 * t >= ke) continue;
        float dk, ek;
        sel_bounds(dv[t], nv[t], c1, c2, dk, ek);
        float u = dk + ek;
#pragma unroll
        for (int a = 0; a < MAX_MA; ++a) {
          if (a < ma && u < best[a]) { const float tt = best[a]; best[a] = u; u = tt; }
        }
      }
    }
    // the wave's ma smallest upper bounds, ascending
    int head = 0;
    for (int a = 0; a < ma; ++a) {
      float v = INFINITY;
#pragma unroll
      for (int q = 0; q < MAX_MA; ++q)
        if (q == head) v = best[q];
      float m = v;
      int who = lane;
      for (int o = 32; o > 0; o >>= 1) {
        const float om = __shfl_xor(m, o, 64);
        const int ow = __shfl_xor(who, o, 64);
        if (om < m || (om == m && ow < who)) { m = om; who = ow; }
      }
      if (lane == 0) L.wub[wave][a] = m;
      if (lane == who) ++head;
    }
  }
  __syncthreads();
  // U: the ma-th smallest of the (four waves') ascending lists
  float U = INFINITY;
  {
    int h[4] = {0, 0, 0, 0};
    for (int a = 0; a < ma; ++a) {
      int bw = 0;
      float bv = INFINITY;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const bool mine = SPLIT || w == wave;
        const float v = mine && h[w] < ma ? L.wub[w][h[w]] : INFINITY;
        if (v < bv) { bv = v; bw = w; }
      }
      U = bv;
#pragma unroll
      for (int w = 0; w < 4; ++w)
        if (w == bw) ++h[w];
    }
  }
  if (!rescan) {
    // keep this wave's candidates within U, in order (each chunk of 64 is
    // read before any of it is overwritten, and entries only move down)
    int kept = 0;
    for (int q = 0; q * 64 < n_w; ++q) {
      const int c = q * 64 + lane;
      const bool in = c < n_w;
      const int kc = in ? L.wk[wave][c] : 0;
      const bool f = in && L.wlb[wave][c] <= U;
      const unsigned long long bal = __ballot(f);
      if (f) L.wk[wave][kept + __popcll(bal & ((1ull << lane) - 1ull))] = kc;
      kept += __popcll(bal);
    }
    n_w = kept;
  } else {
    // this wave's candidates: d^_k - e_k <= U, in ascending k
    n_w = 0;
    for (int k0 = kb; k0 < ke; k0 += 64 * SEL_UNROLL) {
      float dv[SEL_UNROLL], nv[SEL_UNROLL];
#pragma unroll
      for (int t = 0; t < SEL_UNROLL; ++t) {
        const int k = k0 + 64 * t + lane;
        dv[t] = k < ke ? Dr[k] : 0.f;
        nv[t] = k < ke ? nhi[k] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < SEL_UNROLL; ++t) {
        const int k = k0 + 64 * t + lane;
        bool f = false;
        if (k < ke) {
          float dk, ek;
          sel_bounds(dv[t], nv[t], c1, c2, dk, ek);
          f = dk - ek <= U;
        }
        const unsigned long long bal = __ballot(f);
        const int pos = n_w + __popcll(bal & ((1ull << lane) - 1ull));
        if (f && pos < SEL_CAP) L.wk[wave][pos] = k;
        n_w += __popcll(bal);
      }
    }
  }
  // the candidate list: the waves' lists in wave order (ascending k) when
  // the row is split, else the wave's own; the first SEL_CAP kept
  int n_c = n_w;
  const int* cand = L.wk[wave];
  float* chi = L.chi[wave];
  float* clo = L.clo[wave];
  if (SPLIT) {
    if (lane == 0) L.wn[wave] = n_w;
    __syncthreads();
    int before = 0;
    n_c = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if (w < wave) before += L.wn[w];
      n_c += L.wn[w];
    }
    for (int c = lane; c < min(n_w, SEL_CAP); c += 64)
      if (before + c < SEL_CAP) L.cand[before + c] = L.wk[wave][c];
    cand = L.cand;
    chi = L.chi[0];
    clo = L.clo[0];
  }
  if (n_c > SEL_CAP) {
    if ((SPLIT ? threadIdx.x == 0 : lane == 0) && active) atomicAdd(overflow, 1);
    n_c = SEL_CAP;
  }
  if (SPLIT) __syncthreads();
  // compensated distances of the candidates (split rows: wave w takes
  // candidates w, w + 4, ...), 8 float4 pieces of each row in flight per lane
  for (int c = SPLIT ? wave : 0; c < n_c; c += SPLIT ? 4 : 1) {
    const int k = cand[c];
    const float4* b4 = reinterpret_cast<const float4*>(cb + (int64_t)k * dim);
    float sd = 0.f, cc = 0.f;
    for (int u0 = lane; u0 < n4; u0 += 64 * 8) {
      float4 xa[8], ba[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int u = u0 + 64 * q;
        xa[q] = u < n4 ? x4[u] : make_float4(0.f, 0.f, 0.f, 0.f);
        ba[q] = u < n4 ? b4[u] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        dot2_step(xa[q].x, ba[q].x, sd, cc);
        dot2_step(xa[q].y, ba[q].y, sd, cc);
        dot2_step(xa[q].z, ba[q].z, sd, cc);
        dot2_step(xa[q].w, ba[q].w, sd, cc);
      }
    }
    const ff dot = ff_wave_sum(sd, cc);
    const ff d = ff_add(ff{nhi[k], nlo[k]}, ff{-2.f * dot.hi, -2.f * dot.lo});
    if (lane == 0) { chi[c] = d.hi; clo[c] = d.lo; }
  }
  __syncthreads();
  // the ma smallest by (distance, index): wave 0 for a split row, else each
  // wave for its own
  if (!SPLIT || wave == 0) {
    bool used[SEL_CAP / 64];
#pragma unroll
    for (int q = 0; q < SEL_CAP / 64; ++q) used[q] = false;
    for (int a = 0; a < ma; ++a) {
      float bh = INFINITY, bl = INFINITY;
      int bk = 0x7fffffff, bq = -1;
#pragma unroll
      for (int q = 0; q < SEL_CAP / 64; ++q) {
        const int c = q * 64 + lane;
        if (c < n_c && !used[q]) {
          const int k = cand[c];
          if (dk_less(chi[c], clo[c], k, bh, bl, bk)) {
            bh = chi[c]; bl = clo[c]; bk = k; bq = q;
          }
        }
      }
      int who = lane;
      for (int o = 32; o > 0; o >>= 1) {
        const float oh = __shfl_xor(bh, o, 64), ol = __shfl_xor(bl, o, 64);
        const int ok = __shfl_xor(bk, o, 64), ow = __shfl_xor(who, o, 64);
        if (dk_less(oh, ol, ok, bh, bl, bk)) { bh = oh; bl = ol; bk = ok; who = ow; }
      }
      if (lane == who && bq >= 0) {
#pragma unroll
        for (int q = 0; q < SEL_CAP / 64; ++q)
          if (q == bq) used[q] = true;
      }
      if (lane == 0 && active) {
        // performed where every XCD sees it, like the count: a batch item
        // then needs no release fence, only the wait for its own stores
        __hip_atomic_store(&words[r * ma + a], bk < K ? bk : -1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        if (counts != nullptr && bk < K) atomicAdd(&counts[bk], 1);
      }
    }
  }
  __syncthreads();  // LDS is reused by the next item
}

__global__ __launch_bounds__(256) void assign_select_kernel(
    const float* __restrict__ x, int64_t r0, int64_t r1, const float* __restrict__ cb,
    int K, int dim, int ma, const float* __restrict__ D, const float* __restrict__ nhi,
    const float* __restrict__ nlo, float gamma2, int32_t* __restrict__ words,
    int32_t* __restrict__ overflow) {
  __shared__ __align__(16) uint8_t smem[SEL_LDS];
  select_rows<true>(x, r0, r1, cb, K, dim, ma, D, nhi, nlo, gamma2, words, overflow, nullptr,
                    blockIdx.x, smem);
}

gift_status launch_assign(const float* x, int64_t n, int dim, const float* cb, int K, int ma,
                          int32_t* words, float* D, int64_t chunk_rows, float* nhi, float* nlo,
                          int32_t* overflow, uint8_t* xs, uint8_t* cbs, hipStream_t st) {
  if (n <= 0) return GIFT_OK;
  GIFT_CHECK(xs != nullptr && cbs != nullptr, GIFT_EINVAL, "split-row buffers missing");
  hipLaunchKernelGGL(norms_kernel, dim3((K + 3) / 4), dim3(256), 0, st, cb, K, dim, nhi, nlo);
  GIFT_LAUNCHED();
  const size_t split_lds = Dma2Shape<4, 2, 4, 2>::LDS_BYTES;
  {
    const gift_status s = ensure_dynamic_lds(reinterpret_cast<const void*>(dots_split_kernel), split_lds);
    if (s != GIFT_OK) return s;
  }
  launch_split_rows(cb, K, dim, cbs, st);
  GIFT_LAUNCHED();
  const float gamma2 = assign_gamma2(dim);
  const int64_t nc = (K + SPLIT_TILE - 1) / SPLIT_TILE;
  for (int64_t r0 = 0; r0 < n; r0 += chunk_rows) {
    const int64_t r1 = r0 + chunk_rows < n ? r0 + chunk_rows : n;
    launch_split_rows(x + r0 * dim, r1 - r0, dim, xs, st);
    GIFT_LAUNCHED();
    const int64_t nr = (r1 - r0 + SPLIT_TILE - 1) / SPLIT_TILE;
    hipLaunchKernelGGL(dots_split_kernel, dim3((unsigned)(nr * nc)), dim3(512), split_lds, st, xs,
                       r0, r1, cbs, K, dim, D, nr, nc, nullptr, nullptr, (int64_t)0);
    GIFT_LAUNCHED();
    hipLaunchKernelGGL(assign_select_kernel, dim3((unsigned)(r1 - r0)), dim3(256), 0, st,
                       x, r0, r1, cb, K, dim, ma, D, nhi, nlo, gamma2, words, overflow);
    GIFT_LAUNCHED();
  }
  return GIFT_OK;
}

// ------------------------------------------------------------------ bucket sort
// Stable counting sort of items 0..n-1 by key in [0, K): per-block key
// histograms, a scan over blocks per key, a scan over keys, and an in-order
// scatter by one wave per block.  Items of one key end up in ascending item
// order.  K <= 16384.
constexpr int BK_ITEMS = 4096;

__global__ __launch_bounds__(256) void bucket_count_kernel(const int32_t* __restrict__ keys,
                                                           int64_t n, int K, int nb,
                                                           int32_t* __restrict__ hist) {
  extern __shared__ int cnt[];
  for (int k = threadIdx.x; k < K; k += 256) cnt[k] = 0;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * BK_ITEMS;
  for (int i = threadIdx.x; i < BK_ITEMS; i += 256) {
    const int64_t g = i0 + i;
    if (g < n) {
      const int k = keys[g];
      if (k >= 0 && k < K) atomicAdd(&cnt[k], 1);  // out-of-range keys are dropped
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += 256) hist[(int64_t)k * nb + blockIdx.x] = cnt[k];
}

// hist[k][b] := exclusive prefix over b; totals[k] = row sum.
__global__ __launch_bounds__(256) void bucket_scan_blocks_kernel(int32_t* __restrict__ hist,
                                                                 int K, int nb,
                                                                 int64_t* __restrict__ totals) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= K) return;
  int32_t* h = hist + (int64_t)k * nb;
  int64_t run = 0;
  for (int b = 0; b < nb; ++b) {
    const int32_t v = h[b];
    h[b] = (int32_t)run;
    run += v;
  }
  totals[k] = run;
}

// off[0] = 0, off[k+1] = off[k] + vals[k] (single block).
__global__ __launch_bounds__(1024) void exclusive_scan_kernel(const int64_t* __restrict__ vals,
                                                              int K, int64_t* __restrict__ off) {
  __shared__ int64_t part[1024];
  const int per = (K + 1023) / 1024;
  const int k0 = threadIdx.x * per;
  int64_t s = 0;
  for (int k = k0; k < k0 + per && k < K; ++k) s += vals[k];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - s;
  for (int k = k0; k < k0 + per && k < K; ++k) {
    off[k] = run;
    run += vals[k];
  }
  if (threadIdx.x == 1023) off[K] = part[1023];
}

// In-order scatter by one wave per block, 64 items at a time: a lane's
// item goes after the block's earlier items of its key and after the
// earlier lanes of its chunk with that key (counted with shuffles), and the
// last such lane advances the key's position.  `mode` selects what is
// written per item:
//   0: out_a[pos] = item
//   1: F-IF entries, item e = v * ma + a: out_a = v / n_views (shape),
//      out_b = v % n_views (view)
__global__ __launch_bounds__(64) void bucket_scatter_kernel(
    const int32_t* __restrict__ keys, int64_t n, int K, int nb, const int32_t* __restrict__ hist,
    const int64_t* __restrict__ off, int mode, int ma, int n_views,
    int32_t* __restrict__ out_a, int32_t* __restrict__ out_b) {
  extern __shared__ int32_t pos[];
  const int lane = threadIdx.x;
  for (int k = lane; k < K; k += 64) pos[k] = (int32_t)(off[k] + hist[(int64_t)k * nb + blockIdx.x]);
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * BK_ITEMS;
  const int64_t i1 = i0 + BK_ITEMS < n ? i0 + BK_ITEMS : n;
  for (int64_t c0 = i0; c0 < i1; c0 += 64) {
    const int64_t i = c0 + lane;
    const int k = i < i1 ? keys[i] : -1;
    const bool ok = k >= 0 && k < K;  // out-of-range keys are dropped
    int rank = 0, last = 1;
    for (int j = 0; j < 64; ++j) {
      const int kj = __shfl(k, j, 64);
      if (kj == k) {
        if (j < lane) ++rank;
        if (j > lane) last = 0;
      }
    }
    const int64_t p = ok ? (int64_t)pos[k] + rank : 0;  // < n < 2^31
    __syncthreads();  // every lane has read its key's position
    if (ok) {
      if (mode == 0) {
        out_a[p] = (int32_t)i;
      } else {
        const int64_t v = i / ma;
        out_a[p] = (int32_t)(v / n_views);
        out_b[p] = (int32_t)(v % n_views);
      }
      if (last) pos[k] = (int32_t)p + 1;
    }
    __syncthreads();  // positions advanced before the next chunk reads them
  }
}

size_t bucket_sort_ws(int64_t n, int K) {
  const int64_t nb = (n + BK_ITEMS - 1) / BK_ITEMS;
  return ((size_t)nb * K * 4 + 255) / 256 * 256 + ((size_t)K * 8 + 255) / 256 * 256;
}

gift_status launch_bucket_sort(const int32_t* keys, int64_t n, int K, int64_t* off,
                               int mode, int ma, int n_views, int32_t* out_a, int32_t* out_b,
                               void* ws, hipStream_t st) {
  GIFT_CHECK(K >= 1 && K <= 16384, GIFT_EUNSUPPORTED, "K must be in 1..16384");
  const int64_t nb64 = (n + BK_ITEMS - 1) / BK_ITEMS;
  GIFT_CHECK(n < ((int64_t)1 << 31), GIFT_ECAPACITY, "too many items");
  const int nb = (int)(nb64 > 0 ? nb64 : 1);
  int32_t* hist = static_cast<int32_t*>(ws);
  int64_t* totals = reinterpret_cast<int64_t*>(static_cast<char*>(ws) +
                                               ((size_t)nb * K * 4 + 255) / 256 * 256);
  if (n > 0) {
    hipLaunchKernelGGL(bucket_count_kernel, dim3(nb), dim3(256), (size_t)K * 4, st, keys, n, K,
                       nb, hist);
    GIFT_LAUNCHED();
  } else {
    hipLaunchKernelGGL(bucket_count_kernel, dim3(1), dim3(256), (size_t)K * 4, st, keys, 0, K, 1,
                       hist);
    GIFT_LAUNCHED();
  }
  hipLaunchKernelGGL(bucket_scan_blocks_kernel, dim3((K + 255) / 256), dim3(256), 0, st, hist, K,
                     nb, totals);
  GIFT_LAUNCHED();
  hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(1024), 0, st, totals, K, off);
  GIFT_LAUNCHED();
  if (n > 0) {
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(nb), dim3(64), (size_t)K * 4, st, keys, n, K,
                       nb, hist, off, mode, ma, n_views, out_a, out_b);
    GIFT_LAUNCHED();
  }
  return GIFT_OK;
}

// ------------------------------------------------------------------ k-means
__global__ __launch_bounds__(256) void gather_rows_kernel(const float* __restrict__ x,
                                                          const int64_t* __restrict__ idx,
                                                          int K, int dim, float* __restrict__ out) {
  const int k = blockIdx.y;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < dim; t += gridDim.x * 256)
    out[(int64_t)k * dim + t] = x[idx[k] * dim + t];
}

// Centroid = float64 sum of the members in ascending row order, divided in
// float64, rounded once to float32; an empty cluster keeps its centroid.
__global__ __launch_bounds__(256) void centroid_kernel(const float* __restrict__ x, int dim,
                                                       const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ members,
                                                       const float* __restrict__ old_cb,
                                                       float* __restrict__ new_cb) {
  const int k = blockIdx.y;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= dim) return;
  const int64_t m0 = off[k], m1 = off[k + 1];
  float out;
  if (m1 == m0) {
    out = old_cb[(int64_t)k * dim + t];
  } else {
    double s = 0.0;
    for (int64_t m = m0; m < m1; ++m) s = s + (double)x[(int64_t)members[m] * dim + t];
    out = (float)(s / (double)(m1 - m0));
  }
  new_cb[(int64_t)k * dim + t] = out;
}

__global__ __launch_bounds__(256) void count_changes_kernel(const int32_t* __restrict__ a,
                                                            const int32_t* __restrict__ b,
                                                            int64_t n, int32_t* __restrict__ cnt) {
  __shared__ int part[4];
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    c += a[i] != b[i];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = part[0] + part[1] + part[2] + part[3];
    if (tot) atomicAdd(cnt, tot);
  }
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return;
  const int64_t blocks = (n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

void launch_gather_rows(const float* x, const int64_t* idx, int K, int dim, float* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3((dim + 255) / 256, K), dim3(256), 0, st, x, idx,
                     K, dim, out);
}

void launch_centroids(const float* x, int dim, int K, const int64_t* off, const int32_t* members,
                      const float* old_cb, float* new_cb, hipStream_t st) {
  hipLaunchKernelGGL(centroid_kernel, dim3((dim + 255) / 256, K), dim3(256), 0, st, x, dim, off,
                     members, old_cb, new_cb);
}

void launch_count_changes(const int32_t* a, const int32_t* b, int64_t n, int32_t* cnt,
                          hipStream_t st) {
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(count_changes_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256),
                     0, st, a, b, n, cnt);
}

// ------------------------------------------------------------------ list scan
// tile_off[w+1] - tile_off[w] = ceil(|L_w| / tile_len) list tiles (single block).
__global__ __launch_bounds__(1024) void list_tiles_kernel(const int64_t* __restrict__ off, int K,
                                                          int tile_len,
                                                          int64_t* __restrict__ tcount) {
  for (int w = threadIdx.x; w < K; w += 1024)
    tcount[w] = (off[w + 1] - off[w] + tile_len - 1) / tile_len;
}

// One block per list tile of 128 entries and the batch's query views whose
// word is that list: MFMA dots (entries x query views, 128 x 128 tiles, or
// one 128 x 32 tile for up to 32 query views, 128 x 16 for up to 16 with
// float32 rows), the per-shape maximum over
// the tile's entries (entries of a shape are contiguous), and an atomic max
// into mbuf[query view][shape] (row stride ldn; 0 = no matching view yet).
// Tile b of list w (tile_off[w] <= b < tile_off[w + 1]) holds entries
// [tile_len (b - tile_off[w]), + tile_len) of the list (tile_len <= 128: the
// MFMA tile's rows past it are padding).  Groups of at most narrow_max
// (<= 32) query views take the narrow tile.
// Scales: per-view float32 (BF16 / e4m3) or E8M0 rows (MX), null for float32.
// NARROW_DMA: narrow tiles of whole 128-byte sub-tiles use the
// direct-to-LDS gather pipeline instead of register staging.
// Float32 rows sum each K-tile into a fresh block (MFMA_F32_BLOCKED), so
// every first-pass dot of the scan is within gamma(48 + d / 32 + 2)
// sum |x y| of the exact one.
template <int DT, bool NARROW_DMA = true>
__device__ __forceinline__ void scan_list_tile(
    const uint8_t* __restrict__ db, const void* __restrict__ db_scale_v, int n_views,
    int row_bytes, const int64_t* __restrict__ loff, const int32_t* __restrict__ ent_shape,
    const int32_t* __restrict__ ent_view, const int64_t* __restrict__ tile_off, int w,
    const int64_t* __restrict__ goff, const int32_t* __restrict__ gitems,
    const uint8_t* __restrict__ qv, const void* __restrict__ q_scale_v,
    uint32_t* __restrict__ mbuf, int64_t ldn, int64_t b, uint8_t* lds, int tile_len = 128,
    int narrow_max = 32) {
  using T = TileShape<2, 2>;
  constexpr bool MX = DT == GIFT_MXFP8 || DT == GIFT_MXFP4;
  constexpr bool SCALED = DT == GIFT_BF16 || DT == GIFT_FP8E4M3;
  constexpr int MT = DT == GIFT_F32 ? MFMA_F32_BLOCKED : DT;  // MFMA form of the tiles
  const float* db_scale = static_cast<const float*>(db_scale_v);
  const float* q_scale = static_cast<const float*>(q_scale_v);
  const int64_t g0 = goff[w], g1 = goff[w + 1];
  if (g0 == g1) return;
  const int64_t e0 = loff[w] + (b - tile_off[w]) * tile_len;
  const int64_t e1 = e0 + tile_len < loff[w + 1] ? e0 + tile_len : loff[w + 1];
  const int ne = (int)(e1 - e0);
  float* C = reinterpret_cast<float*>(lds);  // [128][129] after the main loop
  const int wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  // the tile rows' view scales, read once per tile (the main loop's
  // barriers order these writes before the epilogues' reads)
  __shared__ float rscale[128];
  if (SCALED && threadIdx.x < 128 && (int)threadIdx.x < ne) {
    const int64_t en = e0 + threadIdx.x;
    rscale[threadIdx.x] = db_scale[(int64_t)ent_shape[en] * n_views + ent_view[en]];
  }

  // Per-shape maximum over this tile's entries for column c (rows [rbeg,
  // rend) of C, row stride ld), folded into mbuf for query view qi.
  // The entries' shapes are read 8 at a time, all loads in flight, before
  // they are used.
  auto fold = [&](int c, int ld, int rbeg, int rend, int qi) {
    const float cs = SCALED ? q_scale[qi] : 1.f;
    int cur = -1;
    float m = -INFINITY;
    for (int r0 = rbeg; r0 < rend; r0 += 8) {
      int shp8[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) shp8[t] = r0 + t < rend ? ent_shape[e0 + r0 + t] : -1;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (r0 + t < rend) {
          const int shp = shp8[t];
          if (shp != cur) {
            if (cur >= 0) atomicMax(&mbuf[(int64_t)qi * ldn + cur], float_order(m * cs));
            cur = shp;
            m = -INFINITY;
          }
          m = fmaxf(m, C[(r0 + t) * ld + c]);
        }
      }
    }
    if (cur >= 0) atomicMax(&mbuf[(int64_t)qi * ldn + cur], float_order(m * cs));
  };

  if constexpr (!MX) {
    // up to 32 query views: one 128 x 32 tile instead of 128 x 128 mostly
    // padding.  BF16 rows take it only through the direct-to-LDS loop: the
    // register-staged narrow loop gave wrong, run-to-run varying BF16 dots
    // inside the persistent batch kernel, so BF16 rows that are no whole
    // number of 128-byte sub-tiles use the 128 x 128 tiles instead.
    const bool narrow_ok =
        DT != GIFT_BF16 || (NARROW_DMA && row_bytes % DMA2_KSUB == 0);
    if (g1 - g0 <= narrow_max && narrow_ok) {
      using N = NarrowShape;
      f32x16 acc;
      if (NARROW_DMA && row_bytes % DMA2_KSUB == 0) {
        // direct-to-LDS gather, two 128-byte sub-tiles in flight; pad rows
        // read the tile's first entry or query view
        const uint8_t* src[NARROW_NI];
#pragma unroll
        for (int i = 0; i < NARROW_NI; ++i) {
          const int r = narrow_dma_row(i);
          if (r < N::BM) {
            const int64_t e = e0 + (r < ne ? r : 0);
            src[i] = db + ((int64_t)ent_shape[e] * n_views + ent_view[e]) * (int64_t)row_bytes;
          } else {
            const int64_t c = g0 + (r - N::BM);
            src[i] = qv + (int64_t)gitems[c < g1 ? c : g0] * row_bytes;
          }
        }
        if constexpr (DT == GIFT_F32) {
          if (g1 - g0 <= 16) {
            // up to 16 query views: 128 x 16 on 16x16x4 MFMA, 8 rows per segment
            f32x4 acc16[2];
            mfma_tile_mainloop_narrow16_dma_f32(lds, src, row_bytes, acc16);
            constexpr int LD16 = 17;
#pragma unroll
            for (int bk = 0; bk < 2; ++bk)
#pragma unroll
              for (int t = 0; t < 4; ++t)
                C[(wave * 32 + bk * 16 + 4 * ((threadIdx.x & 63) >> 4) + t) * LD16 + (threadIdx.x & 15)] =
                    acc16[bk][t];
            __syncthreads();
            const int c = threadIdx.x & 15, seg = threadIdx.x >> 4;
            if (g0 + c < g1) {
              const int rbeg = seg * 8, rend = rbeg + 8 < ne ? rbeg + 8 : ne;
              fold(c, LD16, rbeg, rend, gitems[g0 + c]);
            }
            __syncthreads();
            return;
          }
        }
        mfma_tile_mainloop_narrow_dma<MT>(lds, src, row_bytes, acc);
      } else {
        const uint8_t* src[N::LOADS];
#pragma unroll
        for (int it = 0; it < N::LOADS; ++it) {
          const int r = staged_row(it);
          const uint8_t* p = nullptr;
          if (r < N::BM) {
            if (r < ne) {
              const int64_t e = e0 + r;
              p = db + ((int64_t)ent_shape[e] * n_views + ent_view[e]) * (int64_t)row_bytes;
            }
          } else if (g0 + (r - N::BM) < g1) {
            p = qv + (int64_t)gitems[g0 + (r - N::BM)] * row_bytes;
          }
          src[it] = p;
        }
        mfma_tile_mainloop_narrow<MT>(lds, src, row_bytes, acc);
      }
      constexpr int LD = N::BN + 1;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = wave * 32 + acc_row(0, e);
        float v = acc[e];
        if (SCALED && r < ne) v *= rscale[r];
        C[r * LD + acc_col(0)] = v;
      }
      __syncthreads();
      // 32 columns x 8 segments of 16 rows
      const int c = threadIdx.x & 31, seg = threadIdx.x >> 5;
      if (g0 + c < g1) {
        const int rbeg = seg * 16, rend = rbeg + 16 < ne ? rbeg + 16 : ne;
        fold(c, LD, rbeg, rend, gitems[g0 + c]);
      }
      __syncthreads();
      return;
    }
  }

  for (int64_t c0 = g0; c0 < g1; c0 += T::BN) {
    const uint8_t* src[T::LOADS];
#pragma unroll
    for (int it = 0; it < T::LOADS; ++it) {
      const int r = staged_row(it);
      const uint8_t* p = nullptr;
      if (r < T::BM) {
        if (r < ne) {
          const int64_t e = e0 + r;
          p = db + ((int64_t)ent_shape[e] * n_views + ent_view[e]) * (int64_t)row_bytes;
        }
      } else {
        const int64_t c = c0 + (r - T::BM);
        if (c < g1) p = qv + (int64_t)gitems[c] * row_bytes;
      }
      src[it] = p;
    }
    f32x16 acc[2][2];
    if constexpr (MX) {
      // E8M0 rows of the entry / query view this lane supplies in each block
      const int nblk = (DT == GIFT_MXFP4 ? 2 * row_bytes : row_bytes) / 32;
      const uint8_t* de8 = static_cast<const uint8_t*>(db_scale_v);
      const uint8_t* qe8 = static_cast<const uint8_t*>(q_scale_v);
      const int l32 = threadIdx.x & 31;
      const uint8_t* sa_row[2];
      const uint8_t* sb_row[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = wr * 64 + i * 32 + l32;
        sa_row[i] = de8;
        if (r < ne)
          sa_row[i] = de8 + ((int64_t)ent_shape[e0 + r] * n_views + ent_view[e0 + r]) * nblk;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t c = c0 + wc * 64 + j * 32 + l32;
        sb_row[j] = c < g1 ? qe8 + (int64_t)gitems[c] * nblk : qe8;
      }
      mfma_tile_mainloop_mx<DT == GIFT_MXFP8 ? 0 : 4, 2, 2>(lds, src, row_bytes, sa_row, sb_row,
                                                            acc);
    } else {
      mfma_tile_mainloop<MT, 2, 2>(lds, src, row_bytes, acc);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int r = wr * 64 + acc_row(i, e);
          const int c = wc * 64 + acc_col(j);
          float v = acc[i][j][e];
          if (SCALED && r < ne) v *= rscale[r];
          C[r * 129 + c] = v;
        }
    __syncthreads();
    {
      const int c = threadIdx.x & 127;
      const int half = threadIdx.x >> 7;
      if (c0 + c < g1) {
        const int rbeg = half * 64, rend = rbeg + 64 < ne ? rbeg + 64 : ne;
        fold(c, 129, rbeg, rend, gitems[c0 + c]);
      }
    }
    __syncthreads();
  }
}

// Tile b of the concatenated lists: finds its list, then as scan_list_tile.
template <int DT>
__device__ __forceinline__ void scan_tile(
    const uint8_t* __restrict__ db, const void* __restrict__ db_scale, int n_views,
    int row_bytes, const int64_t* __restrict__ loff, const int32_t* __restrict__ ent_shape,
    const int32_t* __restrict__ ent_view, const int64_t* __restrict__ tile_off, int K,
    const int64_t* __restrict__ goff, const int32_t* __restrict__ gitems,
    const uint8_t* __restrict__ qv, const void* __restrict__ q_scale,
    uint32_t* __restrict__ mbuf, int64_t ldn, int64_t b, uint8_t* lds) {
  if (b >= tile_off[K]) return;
  // list w with tile_off[w] <= b < tile_off[w+1]
  int lo = 0, hi = K;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tile_off[mid] <= b) lo = mid; else hi = mid;
  }
  scan_list_tile<DT>(db, db_scale, n_views, row_bytes, loff, ent_shape, ent_view, tile_off, lo,
                     goff, gitems, qv, q_scale, mbuf, ldn, b, lds);
}

template <int DT>
__global__ __launch_bounds__(256, 2) void fif_scan_kernel(
    const uint8_t* __restrict__ db, const void* __restrict__ db_scale, int n_views,
    int row_bytes, const int64_t* __restrict__ loff, const int32_t* __restrict__ ent_shape,
    const int32_t* __restrict__ ent_view, const int64_t* __restrict__ tile_off, int K,
    const int64_t* __restrict__ goff, const int32_t* __restrict__ gitems,
    const uint8_t* __restrict__ qv, const void* __restrict__ q_scale,
    uint32_t* __restrict__ mbuf, int64_t ldn) {
  extern __shared__ __align__(16) uint8_t lds[];
  scan_tile<DT>(db, db_scale, n_views, row_bytes, loff, ent_shape, ent_view, tile_off, K, goff,
                gitems, qv, q_scale, mbuf, ldn, blockIdx.x, lds);
}

gift_status launch_fif_scan(const gift_views* db, const int64_t* loff, const int32_t* ent_shape,
                            const int32_t* ent_view, int64_t n_entries, int K,
                            int64_t* tile_off, int64_t* tcount, const int64_t* goff,
                            const int32_t* gitems, const void* qv, const void* qscale,
                            uint32_t* mbuf, int64_t ldn, hipStream_t st) {
  hipLaunchKernelGGL(list_tiles_kernel, dim3(1), dim3(1024), 0, st, loff, K, 128, tcount);
  GIFT_LAUNCHED();
  hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(1024), 0, st, tcount, K, tile_off);
  GIFT_LAUNCHED();
  const int64_t bound = n_entries / 128 + K + 1;
  GIFT_CHECK(bound < ((int64_t)1 << 31), GIFT_ECAPACITY, "too many list tiles");
  static_assert(NARROW_DMA_LDS_BYTES <= 128 * 129 * 4, "the narrow pipeline fits the C tile's LDS");
  const size_t shmem = 128 * 129 * 4;
  const int row_bytes = (int)row_bytes_of(db->dtype, db->dim);
#define GIFT_SCAN_LAUNCH(DTV)                                                                  \
  do {                                                                                         \
    const gift_status s_ = ensure_dynamic_lds(                                                 \
        reinterpret_cast<const void*>(fif_scan_kernel<DTV>), shmem);                           \
    if (s_ != GIFT_OK) return s_;                                                              \
    hipLaunchKernelGGL(fif_scan_kernel<DTV>, dim3((unsigned)bound), dim3(256), shmem, st,      \
                       static_cast<const uint8_t*>(db->data), db->scale, db->n_views,          \
                       row_bytes, loff, ent_shape, ent_view, tile_off, K, goff, gitems,        \
                       static_cast<const uint8_t*>(qv), qscale, mbuf, ldn);                    \
  } while (0)
  switch (db->dtype) {
    case GIFT_F32: GIFT_SCAN_LAUNCH(GIFT_F32); break;
    case GIFT_BF16: GIFT_SCAN_LAUNCH(GIFT_BF16); break;
    case GIFT_FP8E4M3: GIFT_SCAN_LAUNCH(GIFT_FP8E4M3); break;
    case GIFT_MXFP8: GIFT_SCAN_LAUNCH(GIFT_MXFP8); break;
    default: GIFT_SCAN_LAUNCH(GIFT_MXFP4); break;
  }
#undef GIFT_SCAN_LAUNCH
  GIFT_LAUNCHED();
  return GIFT_OK;
}

// S[b][p] = (sum over the query's views of the decoded max, 0 where no view
// of p shares the word) / m, summed in ascending view order.  mbuf rows are
// query views, so each step reads 256 consecutive shapes.
__device__ __forceinline__ float fif_mean(const uint32_t* __restrict__ mbuf, int64_t ldn,
                                          int64_t p, int lo, int hi) {
  float acc = 0.f;
  int i = lo;
  // 16 loads in flight, then 4; the sum stays in ascending view order
  for (; i + 16 <= hi; i += 16) {
    uint32_t u[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) u[t] = mbuf[(int64_t)(i + t) * ldn + p];
#pragma unroll
    for (int t = 0; t < 16; ++t)
      if (u[t] != 0u) acc += order_float(u[t]);
  }
  for (; i + 4 <= hi; i += 4) {
    uint32_t u[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) u[t] = mbuf[(int64_t)(i + t) * ldn + p];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (u[t] != 0u) acc += order_float(u[t]);
  }
  for (; i < hi; ++i) {
    const uint32_t u = mbuf[(int64_t)i * ldn + p];
    if (u != 0u) acc += order_float(u);
  }
  return hi > lo ? acc / (float)(hi - lo) : 0.f;
}

// fif_mean of the 4 consecutive shapes p + 1024 s .. + 3 for s < 4 (those
// below n; n, p and ldn multiples of 4, mbuf 16-byte aligned): 16-byte
// loads, 8 views x 4 of them in flight.  Each shape's sum is taken in
// ascending view order, as in fif_mean, so the results are the same bits.
__device__ __forceinline__ void fif_mean16(const uint32_t* __restrict__ mbuf, int64_t ldn,
                                           int64_t p, int64_t n, int lo, int hi,
                                           float4 (&out)[4]) {
  float acc[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[s][e] = 0.f;
  for (int i = lo; i < hi; i += 8) {
    uint4 u[8][4];
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s)
        u[t][s] = i + t < hi && p + 1024 * s < n
                      ? *reinterpret_cast<const uint4*>(mbuf + (int64_t)(i + t) * ldn + p + 1024 * s)
                      : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (u[t][s].x != 0u) acc[s][0] += order_float(u[t][s].x);
        if (u[t][s].y != 0u) acc[s][1] += order_float(u[t][s].y);
        if (u[t][s].z != 0u) acc[s][2] += order_float(u[t][s].z);
        if (u[t][s].w != 0u) acc[s][3] += order_float(u[t][s].w);
      }
  }
  const float m = (float)(hi - lo);
#pragma unroll
  for (int s = 0; s < 4; ++s)
    out[s] = hi <= lo ? make_float4(0.f, 0.f, 0.f, 0.f)
                      : make_float4(acc[s][0] / m, acc[s][1] / m, acc[s][2] / m, acc[s][3] / m);
}

__global__ __launch_bounds__(256) void reduce_fif_kernel(const uint32_t* __restrict__ mbuf,
                                                         int64_t ldn, int64_t n_shapes,
                                                         const int32_t* __restrict__ qoff,
                                                         float* __restrict__ S) {
  const int b = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n_shapes) return;
  S[(int64_t)b * n_shapes + p] = fif_mean(mbuf, ldn, p, qoff[b], qoff[b + 1]);
}

void launch_reduce_fif(const uint32_t* mbuf, int64_t ldn, int64_t n_shapes, const int32_t* qoff,
                       int n_queries, float* S, hipStream_t st) {
  if (n_shapes <= 0 || n_queries <= 0) return;
  dim3 grid((unsigned)((n_shapes + 255) / 256), (unsigned)n_queries);
  hipLaunchKernelGGL(reduce_fif_kernel, grid, dim3(256), 0, st, mbuf, ldn, n_shapes, qoff, S);
}

// ------------------------------------------------------------------ batch
// One persistent kernel runs the whole first pass of a ragged query batch
// (assign + group + scan + reduce) from a device work queue.  Items are
// numbered phase by phase:
//   Q    split 4 query views (one per wave) for the dot tiles and code
//        them in the storage format
//   GEMM query view x codeword dot tiles (MFMA); each item also clears its
//        share of rows [0, n_v) of mbuf
//   FILL (no items: the clear runs inside the GEMM items)
//   SEL  certified nearest word of one query view (batches of at most
//        BATCH_SEL_SPLIT_MAX views, a whole block per view) or of 4 (one wave
//        each); count views per word
//   PRE  word offsets of the groups and of the active list tiles (one item)
//   SCAT place every query view in its word's group
//   TILE list the tiles of every list whose word has query views
//   SCAN one active list tile against its word's query views
//   RED  per-query mean over its views for BATCH_RED_SHAPES shapes
// The item counts of Q..TILE follow from the batch's view count, which every
// block reads at start; SCAN has one item per active tile (counted by PRE)
// and RED one per (query, shape chunk), so a batch costs what its queries
// touch, not what the plan could hold.  Blocks take items in increasing
// order from an atomic counter.  An item of phase p first waits until every
// item numbered below the first item of p has finished (one `done`
// counter), except that GEMM waits for the Q items alone (a second
// counter); an item at or past the first SCAN
// item first waits for all of Q..TILE, and then knows the SCAN and RED
// ranges.  The items waited for were all taken before by blocks that are
// running, and the earliest unfinished item never waits, so the queue
// always drains.  A wait that
// exceeds its wall-clock limit sets the error word; from then on every wait
// and every item is skipped, so every block exits.
//
// Memory ordering across blocks (the L2 of each XCD is private): every
// wave of an item that produces data for later items waits for its own
// writes, and after the block barrier thread 0 makes them visible at device
// scope (one release fence) before the `done` increment.  A waiting item polls `done` with relaxed
// loads, so the poll does not invalidate caches, and thread 0 takes one
// device-scope acquire fence after the wait, before the block barrier.

__global__ __launch_bounds__(256) void batch_reset_kernel(BatchArgs a) {
  // counters, word counts, and the offsets of unused query slots
  const int n_q = a.desc[0];
  for (int i = threadIdx.x; i < BATCH_CTRL_WORDS; i += 256) a.ctrl[i] = 0ull;
  for (int i = threadIdx.x; i < 2 * BP_END; i += 256) a.phase_ticks[i] = 0ull;
  if (threadIdx.x == 0) a.phase_ticks[2 * BP_END] = (unsigned long long)wall_clock64();
  for (int k = threadIdx.x; k < a.K; k += 256) a.counts[k] = 0;
  if (threadIdx.x == 0) *a.overflow = 0;
  const int32_t last = a.qoff[n_q];
  for (int b = n_q + 1 + threadIdx.x; b <= a.Bmax; b += 256) a.qoff[b] = last;
}

// Thread 0 of a block: waits until *done >= need.  Returns 0, or the error
// word when it is (or becomes) set, or 1 after setting it when the wait
// exceeds `ticks` of the constant-rate wall clock.
__device__ int wait_done(const unsigned long long* done, unsigned long long* err,
                         unsigned long long need, int64_t ticks) {
  const long long t0 = wall_clock64();
  for (int polls = 0;; ++polls) {
    if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) return 0;
    const int e = (int)__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (e != 0) return e;
    if (wall_clock64() - t0 > ticks) {
      __hip_atomic_fetch_or(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 1;
    }
    if (polls < 64) __builtin_amdgcn_s_sleep(2);
    else __builtin_amdgcn_s_sleep(32);
  }
}

// tile_word[b] = the list that tile b of the concatenated lists belongs to.
__global__ __launch_bounds__(256) void tile_word_kernel(const int64_t* __restrict__ tile_off,
                                                        int K, int32_t* __restrict__ tile_word) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  if (w >= K) return;
  for (int64_t b = tile_off[w]; b < tile_off[w + 1]; ++b) tile_word[b] = w;
}

// One wave splits query view v for the codeword GEMM and codes it in the
// storage type for the list scan.
template <int DT>
__device__ __forceinline__ void batch_q_view(const BatchArgs& a, int64_t v) {
  split_row_wave(a.qviews, v, a.dim, a.qsplit);
  if constexpr (DT == GIFT_MXFP8 || DT == GIFT_MXFP4)
    quantize_view_mx_wave(a.qviews, v, a.dim, DT, a.qcodes, static_cast<uint8_t*>(a.qscale));
  else if constexpr (DT != GIFT_F32)
    quantize_view_wave(a.qviews, v, a.dim, DT, a.qcodes, static_cast<float*>(a.qscale));
}

// The Q work outside the persistent kernel: one wave per view of the
// current batch (grid sized for Vmax).
template <int DT>
__global__ __launch_bounds__(256) void batch_q_kernel(BatchArgs a) {
  const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (v < (int64_t)a.desc[1]) batch_q_view<DT>(a, v);
}

// ITEMS: the kernel has the Q and GEMM items (plans that run them in the
// kernels of launch_batch_pre use a copy without them, which needs fewer
// registers).
template <int DT, bool ITEMS>
__global__ __launch_bounds__(256, 2) void fif_batch_kernel(BatchArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ int64_t sh_item;
  __shared__ int64_t sh_nact;
  __shared__ int sh_err;
  // thread 0's per-phase busy ticks and last item end, added to the plan's
  // counters once when the block leaves the queue
  __shared__ unsigned long long sh_busy[BP_END], sh_end[BP_END];
  const int tid = threadIdx.x;
  unsigned long long* head = a.ctrl;
  unsigned long long* done = a.ctrl + 1;
  unsigned long long* err = a.ctrl + 2;
  unsigned long long* n_active_w = a.ctrl + 3;  // active list tiles, written by PRE
  unsigned long long* q_done = a.ctrl + 4;      // finished Q items
  const int n_q = a.desc[0];
  const int64_t n_v = a.desc[1];
  // first items of Q..TILE and of SCAN, from the batch's view count
  int64_t first[BP_SCAN + 1];
  {
    const int64_t n_items[BP_SCAN] = {
        a.ext_gemm ? 0 : (n_v + BATCH_Q_VIEWS - 1) / BATCH_Q_VIEWS,             // Q
        a.ext_gemm ? 0 : ((n_v + 127) / 128) * a.gemm_col_tiles,                // GEMM
        0,  // FILL: the clear runs inside the GEMM items                        // FILL
        n_v <= BATCH_SEL_SPLIT_MAX ? n_v : (n_v + 3) / 4,                       // SEL
        1,                                                                      // PRE
        (n_v + 255) / 256,                                                      // SCAT
        (int64_t)(a.K + 255) / 256};                                            // TILE
    int64_t acc = 0;
#pragma unroll
    for (int i = 0; i < BP_SCAN; ++i) {
      first[i] = acc;
      acc += n_items[i];
    }
    first[BP_SCAN] = acc;
  }
  const int64_t red_chunks = (a.n_shapes + BATCH_RED_SHAPES - 1) / BATCH_RED_SHAPES;
  const int64_t n_red = (int64_t)n_q * red_chunks;
  if (tid < BP_END) { sh_busy[tid] = 0ull; sh_end[tid] = 0ull; }
  int64_t n_active = -1;  // active list tiles, once this block has waited for PRE
  int acquired = -1;      // thread 0: last phase whose inputs this block acquired
  long long t_item = 0;   // thread 0: wall clock once the item's inputs are ready
  for (;;) {
    if (tid == 0) sh_item = (int64_t)atomicAdd(head, 1ull);
    __syncthreads();
    const int64_t item = sh_item;
    __syncthreads();
    int ph;
    int64_t j, need = 0;
    if (item < first[BP_SCAN]) {
      ph = 0;
      while (ph + 1 < BP_SCAN && item >= first[ph + 1]) ++ph;
      j = item - first[ph];
      need = first[ph];
    } else {
      if (n_active < 0) {
        // the SCAN and RED ranges are known once Q..TILE have finished
        if (tid == 0) {
          int e = (int)__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (e == 0) e = wait_done(done, err, (unsigned long long)first[BP_SCAN], a.wait_ticks);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          acquired = BP_SCAN;
          sh_nact = e == 0 ? (int64_t)__hip_atomic_load(n_active_w, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                           : 0;
        }
        __syncthreads();
        n_active = sh_nact;
      }
      if (item < first[BP_SCAN] + n_active) {
        ph = BP_SCAN;
        j = item - first[BP_SCAN];
      } else if (item < first[BP_SCAN] + n_active + n_red) {
        ph = BP_RED;
        j = item - first[BP_SCAN] - n_active;
        need = first[BP_SCAN] + n_active;
      } else {
        break;
      }
    }
    // GEMM reads the views Q split; later phases read what all earlier
    // phases wrote
    const bool needs_wait = ph == BP_GEMM || ph == BP_SEL || ph == BP_PRE || ph == BP_SCAT ||
                            ph == BP_TILE || ph == BP_RED;
    if (tid == 0) {
      int e = (int)__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // phases only grow within a block: one wait and one acquire per phase
      if (needs_wait && ph > acquired && e == 0) {
        // GEMM waits for the Q items alone: they precede it in the queue but
        // may finish after FILL items, which wait for nothing
        e = ph == BP_GEMM ? wait_done(q_done, err, (unsigned long long)first[BP_GEMM], a.wait_ticks)
                          : wait_done(done, err, (unsigned long long)need, a.wait_ticks);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        acquired = ph;
      }
      sh_err = e;
      t_item = wall_clock64();
    }
    __syncthreads();
    // whether the item stored data that later items read with plain loads
    bool wrote = false;
    if (!sh_err) {
      switch (ph) {
        case BP_Q: {
          if constexpr (!ITEMS) break;
          const int wave = tid >> 6;
          for (int64_t v = j * BATCH_Q_VIEWS + wave; v < (j + 1) * BATCH_Q_VIEWS && v < n_v; v += 4)
            batch_q_view<DT>(a, v);
          wrote = true;
          break;
        }
        case BP_GEMM: {
          if constexpr (!ITEMS) break;
          // this item's share of clearing rows [0, n_v) of mbuf, stores that
          // drain while the tile's MFMAs run (the release fence at the end of
          // the item covers them)
          {
            const int64_t n_gemm = ((n_v + 127) / 128) * a.gemm_col_tiles;
            const int64_t lim = n_v * a.n_shapes;
            const int64_t per = ((lim + n_gemm - 1) / n_gemm + 1023) / 1024 * 1024;
            const int64_t e0 = j * per, e1 = e0 + per < lim ? e0 + per : lim;
            for (int64_t e = e0 + 4 * tid; e < e1; e += 1024) {
              if (e + 4 <= e1)
                *reinterpret_cast<uint4*>(a.mbuf + e) = make_uint4(0u, 0u, 0u, 0u);
              else
                for (int64_t t = e; t < e1; ++t) a.mbuf[t] = 0u;
            }
          }
          const int64_t rt = j / a.gemm_col_tiles;
          dots_split_tile(a.qsplit, n_v, a.cbsplit, a.K, a.dim, a.D, rt,
                          j - rt * a.gemm_col_tiles, lds);
          wrote = true;
          break;
        }
        case BP_SEL:
          // writes only through device-scope atomics (the word, its count)
          if (n_v <= BATCH_SEL_SPLIT_MAX)
            select_rows<true>(a.qviews, 0, n_v, a.cb, a.K, a.dim, 1, a.D, a.nhi, a.nlo,
                              a.gamma2, a.qwords, a.overflow, a.counts, j, lds);
          else
            select_rows<false>(a.qviews, 0, n_v, a.cb, a.K, a.dim, 1, a.D, a.nhi, a.nlo,
                               a.gamma2, a.qwords, a.overflow, a.counts, j, lds);
          break;
        case BP_PRE: {
          // group offsets (goff) and active-tile offsets (act_off) over
          // words.  Wave w covers a contiguous range of words, 64
          // consecutive words per step (coalesced loads, 8 steps' loads in
          // flight): pass 1 sums the range, the four wave sums are scanned
          // through LDS, pass 2 scans each step across the wave (shuffles)
          // and writes the offsets with coalesced stores.
          int64_t* wsum = reinterpret_cast<int64_t*>(lds);  // [4] + [4]
          const int lane = tid & 63, wave = tid >> 6;
          const int span = ((a.K + 255) / 256) * 64;  // words per wave
          const int w0 = wave * span, w1 = w0 + span < a.K ? w0 + span : a.K;
          auto load8 = [&](int k0, int (&c)[8], int64_t (&tl)[8]) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int kk = k0 + 64 * q + lane;
              c[q] = kk < w1 ? a.counts[kk] : 0;
              tl[q] = kk < w1 ? a.tile_off[kk + 1] - a.tile_off[kk] : 0;
            }
          };
          int64_t sum = 0, tsum = 0;
          for (int k0 = w0; k0 < w1; k0 += 512) {
            int c[8];
            int64_t tl[8];
            load8(k0, c, tl);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              sum += c[q];
              if (c[q] > 0) tsum += tl[q];
            }
          }
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) {
            sum += __shfl_xor(sum, o, 64);
            tsum += __shfl_xor(tsum, o, 64);
          }
          if (lane == 0) { wsum[wave] = sum; wsum[4 + wave] = tsum; }
          __syncthreads();
          int64_t run = 0, trun = 0;
          for (int w = 0; w < wave; ++w) { run += wsum[w]; trun += wsum[4 + w]; }
          if (tid == 0) {
            a.goff[a.K] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
            // read with an atomic load by every block entering the scan
            // range: published the same way as the queue counters
            __hip_atomic_store(n_active_w, (unsigned long long)(wsum[4] + wsum[5] + wsum[6] + wsum[7]),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          for (int k0 = w0; k0 < w1; k0 += 512) {
            int c[8];
            int64_t tl[8];
            load8(k0, c, tl);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              const int kk = k0 + 64 * q + lane;
              const int64_t x = c[q], t = c[q] > 0 ? tl[q] : 0;
              int64_t xi = x, ti = t;
#pragma unroll
              for (int o = 1; o < 64; o <<= 1) {
                const int64_t px = __shfl_up(xi, o, 64), pt = __shfl_up(ti, o, 64);
                if (lane >= o) { xi += px; ti += pt; }
              }
              if (kk < w1) {
                a.goff[kk] = run + xi - x;
                a.act_off[kk] = (int32_t)(trun + ti - t);
                a.fillc[kk] = 0;
              }
              run += __shfl(xi, 63, 64);
              trun += __shfl(ti, 63, 64);
            }
          }
          wrote = true;
          break;
        }
        case BP_SCAT:
          for (int64_t v = j * 256 + tid; v < j * 256 + 256 && v < n_v; v += 256) {
            const int w = a.qwords[v];
            if (w >= 0 && w < a.K) a.gitems[a.goff[w] + atomicAdd(&a.fillc[w], 1)] = (int32_t)v;
          }
          wrote = true;
          break;
        case BP_TILE: {
          const int w = (int)(j * 256) + tid;
          if (w < a.K && a.counts[w] > 0) {
            const int64_t b0 = a.tile_off[w], b1 = a.tile_off[w + 1];
            int32_t* dst = a.act_tile + a.act_off[w];
            for (int64_t b = b0; b < b1; ++b) dst[b - b0] = (int32_t)b;
          }
          wrote = true;
          break;
        }
        case BP_SCAN: {
          const int64_t b = a.act_tile[j];
          // the list scan of gift_query_fif: same tiles, same products and
          // order, so the same first-pass scores
          scan_list_tile<DT, true>(a.db, a.db_scale, a.n_views, a.row_bytes, a.loff, a.ent_shape,
                             a.ent_view, a.tile_off, a.tile_word[b], a.goff, a.gitems,
                             DT == GIFT_F32 ? reinterpret_cast<const uint8_t*>(a.qviews)
                                            : a.qcodes,
                             a.qscale, a.mbuf, a.n_shapes, b, lds, a.tile_len, a.narrow_max);
          break;
        }
        case BP_RED: {
          // BATCH_RED_SHAPES shapes of one query of the batch
          const int b = (int)(j / red_chunks);
          const int64_t lim = (int64_t)n_v;
          const int lo = (int)(a.qoff[b] < 0 ? 0 : (a.qoff[b] > lim ? lim : a.qoff[b]));
          const int hi = (int)(a.qoff[b + 1] < lo ? lo : (a.qoff[b + 1] > lim ? lim : a.qoff[b + 1]));
          const int64_t p0 = (j - (int64_t)b * red_chunks) * BATCH_RED_SHAPES;
          const bool vec = (a.n_shapes & 3) == 0 &&
                           ((reinterpret_cast<uintptr_t>(a.mbuf) | reinterpret_cast<uintptr_t>(a.S)) & 15) == 0;
          static_assert(BATCH_RED_SHAPES == 4 * 4 * 256, "four float4s of shapes per thread");
          if (vec) {
            // 4 consecutive shapes per thread in each of the item's 4 runs
            // of 1,024 shapes
            const int64_t p = p0 + 4 * tid;
            float4 m4[4];
            fif_mean16(a.mbuf, a.n_shapes, p, a.n_shapes, lo, hi, m4);
#pragma unroll
            for (int s = 0; s < 4; ++s)
              if (p + 1024 * s < a.n_shapes)
                *reinterpret_cast<float4*>(a.S + (int64_t)b * a.n_shapes + p + 1024 * s) = m4[s];
          } else {
            for (int64_t p = p0 + tid; p < p0 + BATCH_RED_SHAPES && p < a.n_shapes; p += 256)
              a.S[(int64_t)b * a.n_shapes + p] = fif_mean(a.mbuf, a.n_shapes, p, lo, hi);
          }
          break;
        }
        default:
          break;
      }
    }
    // Release what later items read with plain loads.  Every wave waits
    // until its own stores and atomics have been performed (vmcnt 0); after
    // the barrier (a workgroup-scope release and acquire) thread 0 alone
    // takes the device-scope release fence, which is cumulative: it covers
    // the whole block's writes with one L2 write-back instead of one per
    // wave.  The word selection and the list scan write only through
    // device-scope atomics, which are performed where every XCD sees them
    // (as the queue counters are), so they need no fence.  The per-query
    // means are read only after the kernel.
    if (wrote || ph == BP_SCAN || ph == BP_SEL) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (tid == 0) {
      if (wrote) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (ph == BP_Q) __hip_atomic_fetch_add(q_done, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // no item waits for RED items, so they skip the shared counter
      if (ph != BP_RED) __hip_atomic_fetch_add(done, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long t_end = (unsigned long long)wall_clock64();
      sh_busy[ph] += t_end - (unsigned long long)t_item;
      if (t_end > sh_end[ph]) sh_end[ph] = t_end;
    }
  }
  if (tid == 0) {
    for (int i = 0; i < BP_END; ++i) {
      if (sh_end[i] == 0ull) continue;
      __hip_atomic_fetch_add(&a.phase_ticks[i], sh_busy[i], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_max(&a.phase_ticks[BP_END + i], sh_end[i], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

void launch_batch_reset(const BatchArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, st, a);
}

gift_status launch_batch_pre(const BatchArgs& a, int dtype, hipStream_t st) {
  const unsigned qgrid = (unsigned)((a.Vmax + 3) / 4);
  switch (dtype) {
    case GIFT_F32: hipLaunchKernelGGL(batch_q_kernel<GIFT_F32>, dim3(qgrid), dim3(256), 0, st, a); break;
    case GIFT_BF16: hipLaunchKernelGGL(batch_q_kernel<GIFT_BF16>, dim3(qgrid), dim3(256), 0, st, a); break;
    case GIFT_FP8E4M3:
      hipLaunchKernelGGL(batch_q_kernel<GIFT_FP8E4M3>, dim3(qgrid), dim3(256), 0, st, a);
      break;
    case GIFT_MXFP8: hipLaunchKernelGGL(batch_q_kernel<GIFT_MXFP8>, dim3(qgrid), dim3(256), 0, st, a); break;
    case GIFT_MXFP4: hipLaunchKernelGGL(batch_q_kernel<GIFT_MXFP4>, dim3(qgrid), dim3(256), 0, st, a); break;
    default: return fail(GIFT_EUNSUPPORTED, "unsupported storage type");
  }
  GIFT_LAUNCHED();
  const size_t split_lds = Dma2Shape<4, 2, 4, 2>::LDS_BYTES;
  {
    const gift_status s = ensure_dynamic_lds(reinterpret_cast<const void*>(dots_split_kernel), split_lds);
    if (s != GIFT_OK) return s;
  }
  const int64_t nr = (a.Vmax + SPLIT_TILE - 1) / SPLIT_TILE;
  const int64_t nc = (a.K + SPLIT_TILE - 1) / SPLIT_TILE;
  hipLaunchKernelGGL(dots_split_kernel, dim3((unsigned)(nr * nc)), dim3(512), split_lds, st,
                     a.qsplit, (int64_t)0, a.Vmax, a.cbsplit, a.K, a.dim, a.D, nr, nc, a.desc + 1,
                     a.mbuf, a.n_shapes);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

gift_status launch_fif_batch(const BatchArgs& a, int dtype, int grid, hipStream_t st) {
  const size_t shmem = 128 * 129 * 4;  // the largest phase: the scan's C tile
  static_assert(SEL_LDS <= 128 * 129 * 4, "word selection fits the batch kernel's LDS");
#define GIFT_BATCH_LAUNCH_1(DTV, IT)                                                           \
  do {                                                                                         \
    const gift_status s_ = ensure_dynamic_lds(                                                 \
        reinterpret_cast<const void*>(fif_batch_kernel<DTV, IT>), shmem);                      \
    if (s_ != GIFT_OK) return s_;                                                              \
    hipLaunchKernelGGL((fif_batch_kernel<DTV, IT>), dim3(grid), dim3(256), shmem, st, a);      \
  } while (0)
#define GIFT_BATCH_LAUNCH(DTV)                                                                 \
  do {                                                                                         \
    if (a.ext_gemm) GIFT_BATCH_LAUNCH_1(DTV, false);                                           \
    else GIFT_BATCH_LAUNCH_1(DTV, true);                                                       \
  } while (0)
  switch (dtype) {
    case GIFT_F32: GIFT_BATCH_LAUNCH(GIFT_F32); break;
    case GIFT_BF16: GIFT_BATCH_LAUNCH(GIFT_BF16); break;
    case GIFT_FP8E4M3: GIFT_BATCH_LAUNCH(GIFT_FP8E4M3); break;
    case GIFT_MXFP8: GIFT_BATCH_LAUNCH(GIFT_MXFP8); break;
    default: GIFT_BATCH_LAUNCH(GIFT_MXFP4); break;
  }
#undef GIFT_BATCH_LAUNCH
#undef GIFT_BATCH_LAUNCH_1
  GIFT_LAUNCHED();
  return GIFT_OK;
}

void launch_tile_word(const int64_t* tile_off, int K, int32_t* tile_word, hipStream_t st) {
  hipLaunchKernelGGL(tile_word_kernel, dim3((K + 255) / 256), dim3(256), 0, st, tile_off, K,
                     tile_word);
}

gift_status launch_norms(const float* cb, int K, int dim, float* nhi, float* nlo, hipStream_t st) {
  hipLaunchKernelGGL(norms_kernel, dim3((K + 3) / 4), dim3(256), 0, st, cb, K, dim, nhi, nlo);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

gift_status launch_list_tiles(const int64_t* loff, int K, int tile_len, int64_t* tcount,
                              int64_t* tile_off, hipStream_t st) {
  hipLaunchKernelGGL(list_tiles_kernel, dim3(1), dim3(1024), 0, st, loff, K, tile_len, tcount);
  GIFT_LAUNCHED();
  hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(1024), 0, st, tcount, K, tile_off);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

// Twice (d^_k carries -2 x.b_k) the split-BF16 dot bound of the GEMM,
// per unit of ||x|| ||b_k||.
float assign_gamma2(int dim) {
  const double u = 5.9604644775390625e-08, nn = 6.0 * 17 + dim / 32 + 2;
  return (float)(2.0 * (3.02 / 65536.0 + 1.02 * (nn * u / (1 - nn * u))) * 1.001);
}

}  // namespace gift
