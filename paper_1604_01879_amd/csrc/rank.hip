// Ranking of Eq. 3 / Eq. 4 scores: block-level top-r selection, the exact
// rescore of the candidates and the final (score desc, id asc) order.
#include "bitonic.h"
#include "kernels.h"
#include "mfma_tile.h"
#include "quant.h"

namespace gift {

// ------------------------------------------------------------------ helpers
constexpr int SEL_THREADS = 512;          // threads of a top-r selection block
constexpr int SEL_WAVES = SEL_THREADS / 64;
constexpr int SEL_UNROLL = 8;             // independent loads in flight per thread

// Exclusive prefix count of `flag` over the threads of a block, in thread
// order; returns the block total through `total`.
__device__ inline int block_excl_count(bool flag, int* wsum, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long bal = __ballot(flag);
  const int in_wave = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wsum[wave] = __popcll(bal);
  __syncthreads();
  int before = 0;
  total = 0;
  for (int w = 0; w < SEL_WAVES; ++w) {
    if (w < wave) before += wsum[w];
    total += wsum[w];
  }
  __syncthreads();
  return before + in_wave;
}

// Bitonic sort of `n` (power of two, <= 4096) 64-bit keys in LDS, ascending.
__device__ inline void bitonic_sort_u64(uint64_t* key, int n) {
  block_bitonic_sort(
      key, n, [](uint64_t a, uint64_t b) { return a < b; },
      [](uint64_t v, int j) { return (uint64_t)__shfl_xor((unsigned long long)v, j, 64); });
}

// ------------------------------------------------------------------ top-r
// Key of (score desc, id asc): complement of the order-preserving bits.
__device__ inline uint32_t desc_key(float s) { return ~float_order(s); }

constexpr int MAX_R = 1024;

// One block per query row; rows b >= *active are skipped (active may be
// null).  Radix selection of the r-th smallest key, 8 bits per pass, with
// SEL_UNROLL coalesced loads in flight per thread, then the collection of
// the r keys and a bitonic sort.  Scores share their high bits, so the
// digit histogram has SEL_HCOPIES copies (lane l counts into copy l %
// SEL_HCOPIES, rows padded against bank conflicts): at most 64 /
// SEL_HCOPIES lanes of a wave add to one counter at once.
constexpr int SEL_HCOPIES = 16;
constexpr int SEL_HLD = 257;  // counters per copy: 256 digits + 1 pad

// Shared memory of a selection block.
struct SelShared {
  uint32_t hist[SEL_HCOPIES * SEL_HLD];
  uint32_t prefix, need, eq;
  int wsum[SEL_WAVES];
  int cnt_less;
  uint64_t keys[MAX_R];
};

// The r smallest (key, id) of row[0, n), id = id0 + index, sorted into
// sh.keys[0, r) (padded with ~0 when n < r).  Block-wide: every thread of
// the block calls it.
__device__ void select_block(const float* __restrict__ row, int64_t n, int64_t id0, int r,
                             SelShared& sh) {
  const int tid = threadIdx.x;
  uint32_t* my_hist = sh.hist + (tid % SEL_HCOPIES) * SEL_HLD;
  constexpr int64_t STRIDE = (int64_t)SEL_THREADS * SEL_UNROLL;
  auto finish = [&](int cnt) {  // sort the cnt gathered keys
    int np2 = 1;
    while (np2 < cnt || np2 < r) np2 <<= 1;
    for (int i = cnt + tid; i < np2; i += SEL_THREADS) sh.keys[i] = ~0ull;
    __syncthreads();
    bitonic_sort_u64(sh.keys, np2);
  };
  if (n <= r) {  // every element
    for (int64_t i = tid; i < n; i += SEL_THREADS)
      sh.keys[i] = ((uint64_t)desc_key(row[i]) << 32) | (uint32_t)(id0 + i);
    __syncthreads();
    finish((int)n);
    return;
  }

  uint32_t prefix = 0, mask = 0, need = (uint32_t)r;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    for (int i = tid; i < SEL_HCOPIES * SEL_HLD; i += SEL_THREADS) sh.hist[i] = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += STRIDE) {
      uint32_t kk[SEL_UNROLL];
#pragma unroll
      for (int u = 0; u < SEL_UNROLL; ++u) {
        const int64_t i = base + u * SEL_THREADS + tid;
        kk[u] = i < n ? desc_key(row[i]) : 0u;
      }
#pragma unroll
      for (int u = 0; u < SEL_UNROLL; ++u) {
        const int64_t i = base + u * SEL_THREADS + tid;
        if (i < n && (kk[u] & mask) == prefix) atomicAdd(&my_hist[(kk[u] >> shift) & 255u], 1u);
      }
    }
    __syncthreads();
    // fold the copies into copy 0
    for (int d = tid; d < 256; d += SEL_THREADS) {
      uint32_t t = 0;
      for (int c = 0; c < SEL_HCOPIES; ++c) t += sh.hist[c * SEL_HLD + d];
      sh.hist[d] = t;
    }
    __syncthreads();
    // The digit of the need-th key: an inclusive scan of the 256 counts
    // (digit d on thread d of the first four waves), then the one digit
    // whose range (excl, incl] holds need, i.e. the first digit whose
    // running count reaches need.
    uint32_t h = 0, incl = 0;
    if (tid < 256) {
      const int lane = tid & 63;
      h = sh.hist[tid];
      incl = h;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, o, 64);
        if (lane >= o) incl += v;
      }
      if (lane == 63) sh.wsum[tid >> 6] = (int)incl;
    }
    __syncthreads();
    if (tid < 256) {
      for (int w = 0; w < (tid >> 6); ++w) incl += (uint32_t)sh.wsum[w];
      const uint32_t excl = incl - h;
      // (thread 255 also when the counts fall short, as a sequential walk
      // would end on the last digit; the counts always reach need)
      if ((excl < need && need <= incl) || (tid == 255 && incl < need)) {
        sh.need = need - excl;
        sh.prefix = prefix | ((uint32_t)tid << shift);
        sh.eq = h;  // after the last pass: the keys equal to the r-th
      }
    }
    __syncthreads();
    need = sh.need;
    prefix = sh.prefix;
    mask |= 255u << shift;
    __syncthreads();
  }
  // `prefix` is the r-th smallest key; take every smaller key and the
  // `need` lowest ids among the keys equal to it.
  if (tid == 0) sh.cnt_less = 0;
  __syncthreads();
  const int n_less = r - (int)need;
  const int n_eq = (int)sh.eq;
  if (n_less + n_eq <= MAX_R) {
    // few ties: gather every key up to the r-th in any order; the sort by
    // (key, id) puts the lowest ids of the tied keys first
    for (int64_t base = 0; base < n; base += STRIDE) {
      uint32_t kk[SEL_UNROLL];
#pragma unroll
      for (int u = 0; u < SEL_UNROLL; ++u) {
        const int64_t i = base + u * SEL_THREADS + tid;
        kk[u] = i < n ? desc_key(row[i]) : 0xffffffffu;
      }
#pragma unroll
      for (int u = 0; u < SEL_UNROLL; ++u) {
        const int64_t i = base + u * SEL_THREADS + tid;
        if (i < n && kk[u] <= prefix) {
          const int pos = atomicAdd(&sh.cnt_less, 1);
          sh.keys[pos] = ((uint64_t)kk[u] << 32) | (uint32_t)(id0 + i);
        }
      }
    }
    __syncthreads();
    finish(n_less + n_eq);
    return;
  }
  // many ties: the smaller keys, then the tied keys in index order
  int taken_eq = 0;
  for (int64_t base = 0; base < n; base += STRIDE) {
    uint32_t kk[SEL_UNROLL];
#pragma unroll
    for (int u = 0; u < SEL_UNROLL; ++u) {
      const int64_t i = base + u * SEL_THREADS + tid;
      kk[u] = i < n ? desc_key(row[i]) : 0xffffffffu;
    }
#pragma unroll
    for (int u = 0; u < SEL_UNROLL; ++u) {
      const int64_t i = base + u * SEL_THREADS + tid;
      const bool less = i < n && kk[u] < prefix;
      const bool eq = i < n && kk[u] == prefix;
      if (less) {
        const int pos = atomicAdd(&sh.cnt_less, 1);
        sh.keys[pos] = ((uint64_t)kk[u] << 32) | (uint32_t)(id0 + i);
      }
      if (taken_eq < (int)need) {  // block-uniform
        int tot;
        const int pos = block_excl_count(eq, sh.wsum, tot);
        if (eq && taken_eq + pos < (int)need)
          sh.keys[n_less + taken_eq + pos] = ((uint64_t)kk[u] << 32) | (uint32_t)(id0 + i);
        taken_eq += tot;
      }
    }
  }
  __syncthreads();
  finish(r);
}

__device__ __forceinline__ void write_top(const SelShared& sh, int64_t b, int r,
                                          int32_t* __restrict__ out_id, float* __restrict__ out_s) {
  for (int i = threadIdx.x; i < r; i += SEL_THREADS) {
    const uint64_t k = sh.keys[i];
    out_id[b * r + i] = (int32_t)(k & 0xffffffffu);
    out_s[b * r + i] = order_float(~(uint32_t)(k >> 32));
  }
}

__global__ __launch_bounds__(SEL_THREADS) void select_top_kernel(
    const float* __restrict__ S, int64_t n, int r, const int32_t* __restrict__ active,
    int32_t* __restrict__ out_id, float* __restrict__ out_s) {
  __shared__ SelShared sh;
  const int b = blockIdx.x;
  if (active != nullptr && b >= *active) return;
  select_block(S + (int64_t)b * n, n, 0, r, sh);
  write_top(sh, b, r, out_id, out_s);
}

// Long rows: chunk c of row b (grid chunks x queries) keeps its r smallest
// (key, id) in tmp[b][c][0, r); every key of the row's top r is among its
// chunk's top r, so the merge below is exact.
__global__ __launch_bounds__(SEL_THREADS) void select_chunk_kernel(
    const float* __restrict__ S, int64_t n, int64_t chunk, int r, const int32_t* __restrict__ active,
    uint64_t* __restrict__ tmp) {
  __shared__ SelShared sh;
  const int b = blockIdx.y, c = blockIdx.x;
  if (active != nullptr && b >= *active) return;
  const int64_t c0 = (int64_t)c * chunk;
  const int64_t len = n - c0 < chunk ? n - c0 : chunk;
  select_block(S + (int64_t)b * n + c0, len, c0, r, sh);
  uint64_t* dst = tmp + ((int64_t)b * gridDim.x + c) * r;
  for (int i = threadIdx.x; i < r; i += SEL_THREADS) dst[i] = sh.keys[i];
}

// The r smallest of row b's n_keys chunk winners (at most SEL_MERGE_CAP):
// n_keys / r lists of r keys, each sorted ascending by select_chunk_kernel.
// Keys are unique ((key, id) pairs), so a key's rank in the union is its
// position in its own list plus, for every other list, the number of that
// list's keys below it (a binary search); a key of rank < r is written at
// its rank.  This replaces a sort of all the winners by one pass with no
// barrier.  Pad keys (~0, chunks shorter than r) are skipped: the row holds
// more than r scores, so they never rank below r.
constexpr int SEL_MERGE_CAP = 4096;
__global__ __launch_bounds__(SEL_THREADS) void select_merge_kernel(
    const uint64_t* __restrict__ tmp, int n_keys, int r, const int32_t* __restrict__ active,
    int32_t* __restrict__ out_id, float* __restrict__ out_s) {
  __shared__ uint64_t keys[SEL_MERGE_CAP];
  const int b = blockIdx.x;
  if (active != nullptr && b >= *active) return;
  const uint64_t* src = tmp + (int64_t)b * n_keys;
  for (int i = threadIdx.x; i < n_keys; i += SEL_THREADS) keys[i] = src[i];
  __syncthreads();
  const int n_lists = n_keys / r;
  for (int i = threadIdx.x; i < n_keys; i += SEL_THREADS) {
    const uint64_t x = keys[i];
    if (x == ~0ull) continue;
    const int c = i / r;
    int rank = i - c * r;
    for (int c2 = 0; c2 < n_lists && rank < r; ++c2) {
      if (c2 == c) continue;
      const uint64_t* list = keys + (int64_t)c2 * r;
      int lo = 0, hi = r;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (list[mid] < x) lo = mid + 1; else hi = mid;
      }
      rank += lo;
    }
    if (rank < r) {
      out_id[(int64_t)b * r + rank] = (int32_t)(x & 0xffffffffu);
      out_s[(int64_t)b * r + rank] = order_float(~(uint32_t)(x >> 32));
    }
  }
}

// Rows longer than two chunks of 16,384 scores (doubled until the chunk
// winners fit the merge) go through the chunked path.
static int64_t select_chunk_len(int64_t n, int r) {
  int64_t chunk = 16384;
  while (((n + chunk - 1) / chunk) * r > SEL_MERGE_CAP) chunk *= 2;
  return n > 2 * chunk ? chunk : 0;
}

size_t select_top_ws(int64_t n, int n_queries, int r) {
  const int64_t chunk = select_chunk_len(n, r);
  if (chunk == 0 || n_queries <= 0) return 0;
  return (size_t)n_queries * ((n + chunk - 1) / chunk) * r * sizeof(uint64_t);
}

void launch_select_top(const float* S, int64_t n, int n_queries, int r, const int32_t* active,
                       int32_t* out_id, float* out_s, void* tmp, hipStream_t st) {
  if (n_queries <= 0) return;
  const int64_t chunk = select_chunk_len(n, r);
  if (chunk == 0 || tmp == nullptr) {
    hipLaunchKernelGGL(select_top_kernel, dim3(n_queries), dim3(SEL_THREADS), 0, st, S, n, r,
                       active, out_id, out_s);
    return;
  }
  const int n_chunks = (int)((n + chunk - 1) / chunk);
  hipLaunchKernelGGL(select_chunk_kernel, dim3(n_chunks, n_queries), dim3(SEL_THREADS), 0, st, S,
                     n, chunk, r, active, static_cast<uint64_t*>(tmp));
  hipLaunchKernelGGL(select_merge_kernel, dim3(n_queries), dim3(SEL_THREADS), 0, st,
                     static_cast<const uint64_t*>(tmp), n_chunks * r, r, active, out_id, out_s);
}

// ------------------------------------------------------------------ rescore
// Pairs handled by block `blk` when the chip runs blocks round-robin over its
// 8 XCDs: XCD x takes the contiguous pair range [x c, x c + c), c = ceil(n / 8),
// so the blocks running together on one XCD (and its L2) share a query.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t blk, int64_t n) {
  const int64_t c = (n + 7) / 8;
  return (blk & 7) * c + (blk >> 3);
}

constexpr int RS_CANDS = 4;                         // candidates per rescore block, one wave each
constexpr int RS_THREADS = 64 * RS_CANDS;
constexpr int RS_ROWS = 64 * (RS_CANDS + 1);        // staged rows: candidate views, then query views
constexpr int RS_PIECES = RS_ROWS * 8 / RS_THREADS;  // 16-byte pieces per thread per K-tile

// First-pass pruning.  Candidates come sorted by first-pass score (desc),
// and each first-pass score is within e_b = (first_err + gamma_(m_b + 2)) *
// 1.001 of the exact score (first_err: the storage bound for unit-norm
// views, the same bound the completeness flag uses).  The k best candidates
// all score at least T = first[k - 1] - e_b exactly, so a candidate with
// first + e_b below T (less a relative 2.4e-7, which absorbs the float
// rounding here and the rescore's own error) cannot be in the top k: it is
// neither staged nor rescored and is ranked last.  Sorted order makes the
// surviving candidates a prefix.  Storage with a loose bound (e4m3, MX)
// prunes nothing.
__device__ __forceinline__ bool first_pass_live(const float* first_row, int c, int k, int m,
                                                float first_err) {
  const float nm = (float)(m + 2) * 5.96046448e-08f;
  const float eb = (first_err + nm / (1.f - nm)) * 1.001f;
  const float T = first_row[k - 1] - eb;
  return first_row[c] + eb >= T - fabsf(T) * 2.4e-7f;
}

// Approximate maximum and near-maximum mask of one query view (this lane's
// column i of block cj) from a wave's 64 x 64 dot tile acc[bi][cj]
// (candidate views in rows, query views in columns): the maximum over the
// views `allowed` to pair with it, and bit j set for every allowed view
// within 2 dot_err of that maximum.  Returns the maximum (-inf when no view
// is allowed) and, through `bits`, the mask (valid in every lane).
__device__ __forceinline__ float view_max_mask(const f32x16 (&acc)[2][2], int cj,
                                               unsigned long long allowed, float dot_err,
                                               unsigned long long& bits) {
  const int half = (threadIdx.x & 63) >> 5;
  float mx = -INFINITY;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int j = bi * 32 + 8 * (e >> 2) + 4 * half + (e & 3);
      if ((allowed >> j) & 1ull) mx = fmaxf(mx, acc[bi][cj][e]);
    }
  mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
  bits = 0ull;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int j = bi * 32 + 8 * (e >> 2) + 4 * half + (e & 3);
      if (((allowed >> j) & 1ull) && acc[bi][cj][e] >= mx - 2.f * dot_err) bits |= 1ull << j;
    }
  const unsigned lo_b = (unsigned)bits, hi_b = (unsigned)(bits >> 32);
  bits |= (unsigned long long)__shfl_xor(lo_b, 32, 64) |
          ((unsigned long long)__shfl_xor(hi_b, 32, 64) << 32);
  return mx;
}

// Views of a candidate (words vw[j * ma + a] of its view j) that may pair
// with query view wq under Eq. 4; every view under Eq. 3 (qwords null).
__device__ __forceinline__ unsigned long long allowed_views(const int32_t* vw, int n_views, int ma,
                                                            bool eq4, int wq) {
  if (!eq4) return n_views >= 64 ? ~0ull : (1ull << n_views) - 1ull;
  unsigned long long a = 0ull;
  for (int j = 0; j < n_views; ++j)
    for (int a2 = 0; a2 < ma; ++a2)
      if (vw[j * ma + a2] == wq) a |= 1ull << j;
  return a;
}

// Candidate rescore, phase 1 (rescore_mask_kernel): one block (four waves)
// per (query, 4 consecutive candidates), blocks in XCD-contiguous order, so
// the query's rows are staged once for four candidates and the blocks
// sharing an XCD share the query.  Approximate dot products of each
// candidate's views (rows) with up to 64 query views (columns) on MFMA;
// wave w owns candidate w, as 2 x 2 blocks of 32 x 32.  Each float32 value
// is split as hi + lo + r (hi, lo bfloat16, |r| <= 2^-16 |x|) and the dot is
// hi.hi' + hi.lo' + lo.hi' on BF16 MFMA (products exact in float32), missing
// at most about 3 * 2^-16 sum |x y|.  Each 32-value K-tile is accumulated
// into a fresh register block and added into a running total, which bounds
// the float32 accumulation depth; dot_err bounds both.  For query view i of
// chunk `it` (views q0 + 64 it + i) the kernel writes the mask of views
// within 2 dot_err of the approximate maximum (bit j of mask[c][q0 + 64 it +
// i], candidate slot c) and the chunk's sum of approximate maxima
// s1[c][q0 + 64 it].
// With `qwords` set (Eq. 4), the pair (q_i, p_j) takes part only when the
// word of q_i is one of the `ma` words of p_j; a query view with no such
// pair gets an empty mask and a maximum of 0.  Only the candidate views that
// share a word with some view of the chunk are staged, compacted (staged row
// r of candidate k is its view cu[k][r], r < nu[k]); the second block of 32
// rows is skipped when at most 32 remain.  Most Eq. 4 candidates match a
// query through a few views, so their rows are read for those views only.
// MODE: RS_FULL, one block per item over the whole K range; RS_PART, block
// (item, split) over K tiles [split kt, (split + 1) kt) of its rows, its
// dot tiles written to `part`; RS_FINISH, one block per item adding the
// n_split partial tiles in split order, then the masks and maxima.  The
// split modes serve batches whose queries have at most 64 views (one
// chunk).  Each split keeps the per-K-tile blocks and running total, and
// the finish adds n_split - 1 more terms, so dot_err bounds them too.
constexpr int RS_FULL = 0, RS_PART = 1, RS_FINISH = 2;

template <int MODE>
__global__ __launch_bounds__(RS_THREADS, 2) void rescore_mask_kernel(
    const float* __restrict__ master, int n_views, int dim,
    const float* __restrict__ qviews, const int32_t* __restrict__ qoff,
    int n_queries, const int32_t* __restrict__ cand, int r, float dot_err,
    const int32_t* __restrict__ qwords, const int32_t* __restrict__ view_words, int ma,
    const int32_t* __restrict__ active, const float* __restrict__ first_s, float first_err,
    int top_k, unsigned long long* __restrict__ mask, float* __restrict__ s1, int64_t ld,
    float* __restrict__ part, int n_split) {
  __shared__ __align__(16) uint8_t lds[RS_ROWS * LROW];
  __shared__ int32_t vw[RS_CANDS][64 * 8];
  __shared__ int32_t qw_chunk[64];
  __shared__ int8_t cu[RS_CANDS][64];
  __shared__ int nu_sh[RS_CANDS];

  const int groups = (r + RS_CANDS - 1) / RS_CANDS;
  const int64_t n_items = (int64_t)(active != nullptr ? *active : n_queries) * groups;
  // With n_split set, the split kernels take batches of at most
  // RESCORE_SPLIT_ITEMS items and this one the larger ones (the same graph
  // serves every batch size up to the plan's capacity).
  if (MODE == RS_FULL && n_split > 1 && n_items <= RESCORE_SPLIT_ITEMS) return;
  if (MODE != RS_FULL && n_items > RESCORE_SPLIT_ITEMS) return;
  int64_t item;
  int split = 0;
  if constexpr (MODE == RS_FULL) {
    item = xcd_contiguous(blockIdx.x, n_items);
  } else if constexpr (MODE == RS_PART) {
    item = blockIdx.x / n_split;
    split = (int)(blockIdx.x - item * n_split);
  } else {
    item = blockIdx.x;
  }
  if (item >= n_items) return;  // past the batch
  const int b = (int)(item / groups);
  const int c0 = (int)(item % groups) * RS_CANDS;
  const int q0 = qoff[b], m = qoff[b + 1] - q0;
  // the block's candidates that survive first-pass pruning (a prefix)
  int n_cand = 0;
  for (int k = 0; k < min(RS_CANDS, r - c0); ++k)
    n_cand += first_pass_live(first_s + (int64_t)b * r, c0 + k, top_k, m, first_err) ? 1 : 0;
  if (n_cand == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, l32 = lane & 31;
  const bool mine = wave < n_cand;  // this wave's candidate exists
  const bool eq4 = qwords != nullptr;
  const int row_bytes = dim * 4;
  const int64_t shape_bytes = (int64_t)n_views * row_bytes;
  const uint8_t* master_b = reinterpret_cast<const uint8_t*>(master);

  // the block's candidate shapes (the last repeated when fewer than 4)
  int64_t shape[RS_CANDS];
#pragma unroll
  for (int k = 0; k < RS_CANDS; ++k) shape[k] = cand[(int64_t)b * r + c0 + min(k, n_cand - 1)];
  const int cslot = c0 + (mine ? wave : 0);

  if (eq4)
#pragma unroll
    for (int k = 0; k < RS_CANDS; ++k)
      for (int x = tid; x < n_views * ma; x += RS_THREADS)
        vw[k][x] = view_words[shape[k] * n_views * ma + x];

  // staging: thread t copies bytes [16 (t & 7), 16 (t & 7) + 16) of each
  // 128-byte K-tile of staged rows (t >> 3) + 32 p, p < RS_PIECES: rows
  // 64 k + r of candidate k (its view cu[k][r]), then 64 RS_CANDS + i of the
  // query chunk, addressed as 32-bit offsets from the row group's base
  uint32_t roff[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
    roff[h] = (uint32_t)((tid >> 3) + 32 * h) * (uint32_t)row_bytes + (uint32_t)(tid & 7) * 16u;
  gptr<uint8_t> gb[RS_CANDS + 1];
#pragma unroll
  for (int k = 0; k < RS_CANDS; ++k) gb[k] = uniform_gptr(master_b + shape[k] * shape_bytes);

  for (int it = 0; it * 64 < m; ++it) {
    if (MODE != RS_FULL && it > 0) break;  // split batches hold queries of at most 64 views
    const int mi = min(64, m - it * 64);
    __syncthreads();  // the previous chunk's epilogue is done with the tables
    if (eq4 && tid < 64) qw_chunk[tid] = tid < mi ? qwords[q0 + it * 64 + tid] : -1;
    __syncthreads();
    {
      // wave k lists candidate k's views that may pair with this chunk
      // (lane j: view j) in ascending order
      bool use = lane < n_views;
      if (use && eq4) {
        bool hit = false;
        for (int a2 = 0; a2 < ma && !hit; ++a2) {
          const int wj = vw[wave][lane * ma + a2];
          for (int i = 0; i < mi; ++i)
            if (qw_chunk[i] == wj) { hit = true; break; }
        }
        use = hit;
      }
      const unsigned long long U = __ballot(use);
      if (use) cu[wave][__popcll(U & ((1ull << lane) - 1ull))] = (int8_t)lane;
      if (lane == 0) nu_sh[wave] = __popcll(U);
    }
    __syncthreads();
    const float* qbase = qviews + (int64_t)(q0 + it * 64) * dim;
    gb[RS_CANDS] = uniform_gptr(reinterpret_cast<const uint8_t*>(qbase));
    unsigned valid = 0u;  // bit p: piece p lies in a present row
#pragma unroll
    for (int p = 0; p < RS_PIECES; ++p) {
      const int g = p >> 1, row = (tid >> 3) + 32 * (p & 1);
      const bool ok = g < RS_CANDS ? (g < n_cand && row < nu_sh[g]) : row < mi;
      valid |= (ok ? 1u : 0u) << p;
    }
    const int nu = nu_sh[wave];
    const bool two = nu > 32;  // the wave's second block of 32 rows has rows
    f32x16 tot[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int cj = 0; cj < 2; ++cj)
#pragma unroll
        for (int e = 0; e < 16; ++e) tot[bi][cj][e] = 0.f;
    // LDS row of a K-tile: 32 high parts (64 bytes) then 32 low parts; lane
    // half h supplies values [16h, 16h + 16) of the tile in two MFMA steps
    const uint8_t* arow = lds + (64 * wave + l32) * LROW + half * 32;
    const uint8_t* brow = lds + (64 * RS_CANDS + l32) * LROW + half * 32;
    uint4 pre[RS_PIECES];
    auto gload = [&](int k0) {
#pragma unroll
      for (int p = 0; p < RS_PIECES; ++p) {
        const int g = p >> 1, row = (tid >> 3) + 32 * (p & 1);
        uint32_t off = roff[p & 1];
        if (g < RS_CANDS)
          off = (uint32_t)cu[g][row & 63] * (uint32_t)row_bytes + (uint32_t)(tid & 7) * 16u;
        pre[p] = (valid >> p) & 1u ? load_at<uint4>(gb[g], off + (uint32_t)k0)
                                   : make_uint4(0, 0, 0, 0);
      }
    };
    // this block's K range (bytes of each row)
    int kb = 0, ke = row_bytes;
    if constexpr (MODE == RS_PART) {
      const int kt = ((row_bytes + 127) / 128 + n_split - 1) / n_split;
      kb = split * kt * 128;
      ke = min(row_bytes, kb + kt * 128);
    }
    if (MODE != RS_FINISH && kb < ke) gload(kb);
    for (int k0 = kb; MODE != RS_FINISH && k0 < ke; k0 += 128) {
      __syncthreads();
#pragma unroll
      for (int p = 0; p < RS_PIECES; ++p) {
        uint2 hi, lo;
        split_bf16x4(pre[p], hi, lo);
        uint8_t* row = lds + ((tid >> 3) + 32 * p) * LROW + (tid & 7) * 8;
        *reinterpret_cast<uint2*>(row) = hi;
        *reinterpret_cast<uint2*>(row + 64) = lo;
      }
      __syncthreads();
      if (k0 + 128 < ke) gload(k0 + 128);  // in flight during the MFMAs
#pragma unroll
      for (int cj = 0; cj < 2; ++cj) {
        uint4 bh[2], bl[2];
#pragma unroll
        for (int st = 0; st < 2; ++st) {
          bh[st] = *reinterpret_cast<const uint4*>(brow + cj * 32 * LROW + st * 16);
          bl[st] = *reinterpret_cast<const uint4*>(brow + cj * 32 * LROW + 64 + st * 16);
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
          if (bi == 1 && !two) continue;  // rows 32..63 hold no view
          uint4 ah[2], al[2];
#pragma unroll
          for (int st = 0; st < 2; ++st) {
            ah[st] = *reinterpret_cast<const uint4*>(arow + bi * 32 * LROW + st * 16);
            al[st] = *reinterpret_cast<const uint4*>(arow + bi * 32 * LROW + 64 + st * 16);
          }
          f32x16 part;
#pragma unroll
          for (int e = 0; e < 16; ++e) part[e] = 0.f;
#pragma unroll
          for (int st = 0; st < 2; ++st) {
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, ah[st]), __builtin_bit_cast(bf16x8, bh[st]), part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, ah[st]), __builtin_bit_cast(bf16x8, bl[st]), part, 0, 0, 0);
            part = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, al[st]), __builtin_bit_cast(bf16x8, bh[st]), part, 0, 0, 0);
          }
#pragma unroll
          for (int e = 0; e < 16; ++e) tot[bi][cj][e] += part[e];
        }
      }
    }
    if constexpr (MODE != RS_FULL) {
      // partial tiles: [item][split][wave][(bi, cj, e)][lane]
      const int64_t slab = (int64_t)RS_CANDS * 64 * 64;
      if constexpr (MODE == RS_PART) {
        float* dst = part + (item * n_split + split) * slab + (int64_t)wave * 64 * 64 + lane;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int cj = 0; cj < 2; ++cj)
#pragma unroll
            for (int e = 0; e < 16; ++e) dst[((bi * 2 + cj) * 16 + e) * 64] = tot[bi][cj][e];
        continue;
      } else {
        for (int sp = 0; sp < n_split; ++sp) {
          const float* src = part + (item * n_split + sp) * slab + (int64_t)wave * 64 * 64 + lane;
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int cj = 0; cj < 2; ++cj)
#pragma unroll
              for (int e = 0; e < 16; ++e) tot[bi][cj][e] += src[((bi * 2 + cj) * 16 + e) * 64];
        }
      }
    }
    float s1_chunk = 0.f;  // this chunk's sum of approximate maxima
#pragma unroll
    for (int cj = 0; cj < 2; ++cj) {
      const int i = cj * 32 + l32;
      const bool live = mine && i < mi;
      unsigned long long allowed =
          allowed_views(vw[wave], n_views, ma, eq4, live && eq4 ? qw_chunk[i] : -1);
      if (eq4) {
        // over the staged rows: row q allowed when its view cu[wave][q] is
        unsigned long long ac = 0ull;
        for (int q = 0; q < nu; ++q) ac |= ((allowed >> cu[wave][q]) & 1ull) << q;
        allowed = live ? ac : 0ull;
      }
      unsigned long long bits;
      const float mx = view_max_mask(tot, cj, allowed, dot_err, bits);
      if (eq4) {
        // staged rows back to views
        unsigned long long vb = 0ull;
        while (bits) {
          const int q = __builtin_ctzll(bits);
          bits &= bits - 1;
          vb |= 1ull << cu[wave][q];
        }
        bits = vb;
      }
      if (half == 0 && live) mask[(int64_t)cslot * ld + q0 + it * 64 + i] = bits;
      float v = (half == 0 && i < mi && mx != -INFINITY) ? mx : 0.f;
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      s1_chunk += v;
    }
    if (mine && lane == 0) s1[(int64_t)cslot * ld + q0 + it * 64] = s1_chunk;
  }
}

// Which candidates can still reach the top k (rescore_mark_kernel, one block
// per query).  s1, the mean of the approximate maxima (the chunk sums
// added in ascending chunk order), is within delta = dot_err + (m + 2)
// 2^-24 1.01 of the exact score (each maximum is within dot_err, plus the
// rounding of the float sum of values below 1 + dot_err).  With T the k-th
// largest s1 - delta, at least k candidates score T or more, so one with
// s1 + delta < T cannot be in the top k; the others are marked for the
// exact evaluation.
__global__ __launch_bounds__(256) void rescore_mark_kernel(
    const float* __restrict__ s1c, int64_t ld, const int32_t* __restrict__ qoff, int r, int k,
    float dot_err, const int32_t* __restrict__ active, const float* __restrict__ first_s,
    float first_err, uint8_t* __restrict__ mark) {
  __shared__ float lb[MAX_R], sv[MAX_R];
  const int b = blockIdx.x;
  if (active != nullptr && b >= *active) return;
  const int q0 = qoff[b], m = qoff[b + 1] - q0;
  const float delta = dot_err + (float)(m + 2) * 5.96046448e-08f * 1.01f;
  const int64_t base = (int64_t)b * r;
  int np2 = 1;
  while (np2 < r) np2 <<= 1;
  for (int i = threadIdx.x; i < np2; i += 256) {
    float v = -INFINITY;
    if (i < r) {
      // a pruned candidate has no approximate score and is never marked
      if (first_pass_live(first_s + base, i, k, m, first_err)) {
        float acc = 0.f;
        for (int it = 0; it * 64 < m; ++it) acc += s1c[(int64_t)i * ld + q0 + it * 64];
        v = m > 0 ? acc / (float)m : 0.f;
      }
      sv[i] = v;
    }
    lb[i] = i < r ? v - delta : -INFINITY;
  }
  __syncthreads();
  // bitonic sort, descending
  block_bitonic_sort(
      lb, np2, [](float a, float b) { return a > b; },
      [](float v, int j) { return __shfl_xor(v, j, 64); });
  const float T = lb[k - 1];
  for (int i = threadIdx.x; i < r; i += 256)
    mark[base + i] = sv[i] != -INFINITY && sv[i] + delta >= T ? 1 : 0;
}

// Candidate rescore, phases 2 and 3 (rescore_exact_kernel): one block (four
// waves) per (query, candidate), blocks in XCD-contiguous order.  Every
// masked pair (q_i, p_j) is re-evaluated with the compensated dot product
// of Ogita, Rump and Oishi (Dot2: error-free products by FMA, error-free
// sums, the errors summed alongside), in float32 arithmetic, and the exact
// maximum over each query view's masked views kept; the block then forms
// the compensated mean over the query views in ascending order.  A query
// view with an empty mask contributes 0.  Lane l takes the float4 pieces
// l, l + 64, ... of both rows, four at a time, summed in four compensated
// chains of at most 16 products (piece k goes to chain k % 4), then across
// the lane's chains and the wave in float-float arithmetic.  The pair (hi,
// lo) is then within about gamma(16)^2 sum |x y| + 16 u^2 sum |x y| of the
// exact dot (about 1e-12 for unit-norm rows at d = 4096).
// Work units pair one candidate view with up to two of the query views
// whose masks hold it, so a view that is the near-maximum of several query
// views (a dozen distinct views cover the 64 query views of a headline
// candidate) is read once per two of them instead of once per query view;
// waves take the units in turn, and each pair's maximum is kept with an
// LDS atomic maximum on its (hi, lo) order key, so the result does not
// depend on the order of the units.
// At 5 waves per SIMD (96 VGPRs, no spills) instead of the 4 that the
// kernel's 102 VGPRs would allow, more units' loads are in flight per CU.
constexpr int EX_BATCH = 4;  // float4 pieces per row per lane in flight per step

__global__ __launch_bounds__(256, 5) void rescore_exact_kernel(
    const float* __restrict__ master, int n_views, int dim,
    const float* __restrict__ qviews, const int32_t* __restrict__ qoff, int n_queries,
    const int32_t* __restrict__ cand, int r, const unsigned long long* __restrict__ mask,
    int64_t ld, const uint8_t* __restrict__ mark, const int32_t* __restrict__ active,
    float* __restrict__ s_hi, float* __restrict__ s_lo) {
  __shared__ float mff_hi[64], mff_lo[64];
  __shared__ unsigned long long msk_s[64];   // the chunk's masks, by query view
  __shared__ unsigned long long best_k[64];  // order key of each query view's maximum
  __shared__ uint32_t units[64 * 33];        // j | i0 << 8 | i1 << 16 (i1 255: none)
  __shared__ int n_units;
  const int64_t n_pairs = (int64_t)(active != nullptr ? *active : n_queries) * r;
  const int64_t pair = xcd_contiguous(blockIdx.x, n_pairs);
  if (pair >= n_pairs) return;  // past the batch
  if (!mark[pair]) {  // cannot reach the top k: ranked last, never returned
    if (threadIdx.x == 0) { s_hi[pair] = -INFINITY; s_lo[pair] = 0.f; }
    return;
  }
  const int b = (int)(pair / r);
  const int q0 = qoff[b], m = qoff[b + 1] - q0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float* pbase = master + (int64_t)cand[pair] * n_views * dim;
  const unsigned long long* pmask = mask + (pair - (int64_t)b * r) * ld + q0;
  const int n4 = dim >> 2;
  ff acc = {0.f, 0.f};
  for (int it = 0; it * 64 < m; ++it) {
    const int mi = min(64, m - it * 64);
    __syncthreads();  // the previous chunk is done with the tables
    if (tid < 64) {
      msk_s[tid] = tid < mi ? pmask[it * 64 + tid] : 0ull;
      best_k[tid] = 0ull;
    }
    if (tid == 0) n_units = 0;
    __syncthreads();
    // units: view j with the query views whose masks hold it, two at a time
    for (int j = wave; j < n_views; j += 4) {
      unsigned long long qm = __ballot(lane < mi && ((msk_s[lane] >> j) & 1ull));
      while (qm) {
        const uint32_t i0 = (uint32_t)__builtin_ctzll(qm);
        qm &= qm - 1;
        uint32_t i1 = 255u;
        if (qm) {
          i1 = (uint32_t)__builtin_ctzll(qm);
          qm &= qm - 1;
        }
        if (lane == 0) units[atomicAdd(&n_units, 1)] = (uint32_t)j | (i0 << 8) | (i1 << 16);
      }
    }
    __syncthreads();
    const int nu = n_units;
    for (int u = wave; u < nu; u += 4) {
      const uint32_t w = units[u];
      const int j = (int)(w & 255u), i0 = (int)((w >> 8) & 255u), i1 = (int)((w >> 16) & 255u);
      const bool two = i1 != 255;  // uniform in the wave
      const gptr<uint8_t> p4 = uniform_gptr(reinterpret_cast<const uint8_t*>(pbase + (int64_t)j * dim));
      const gptr<uint8_t> qa4 = uniform_gptr(
          reinterpret_cast<const uint8_t*>(qviews + (int64_t)(q0 + it * 64 + i0) * dim));
      const gptr<uint8_t> qb4 = uniform_gptr(
          reinterpret_cast<const uint8_t*>(qviews + (int64_t)(q0 + it * 64 + (two ? i1 : i0)) * dim));
      float sa[4] = {0.f, 0.f, 0.f, 0.f}, ca[4] = {0.f, 0.f, 0.f, 0.f};
      float sb[4] = {0.f, 0.f, 0.f, 0.f}, cb[4] = {0.f, 0.f, 0.f, 0.f};
      for (int u0 = lane; u0 < n4; u0 += 64 * EX_BATCH) {
        float4 pa[EX_BATCH], qa[EX_BATCH], qb[EX_BATCH];
#pragma unroll
        for (int k = 0; k < EX_BATCH; ++k) {
          const uint32_t uu = (uint32_t)(u0 + 64 * k);
          const bool in = uu < (uint32_t)n4;
          pa[k] = in ? load_at<float4>(p4, uu * 16u) : make_float4(0.f, 0.f, 0.f, 0.f);
          qa[k] = in ? load_at<float4>(qa4, uu * 16u) : make_float4(0.f, 0.f, 0.f, 0.f);
          qb[k] = in && two ? load_at<float4>(qb4, uu * 16u) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < EX_BATCH; ++k) {
          dot2_step(qa[k].x, pa[k].x, sa[k], ca[k]);
          dot2_step(qa[k].y, pa[k].y, sa[k], ca[k]);
          dot2_step(qa[k].z, pa[k].z, sa[k], ca[k]);
          dot2_step(qa[k].w, pa[k].w, sa[k], ca[k]);
        }
        if (two) {
#pragma unroll
          for (int k = 0; k < EX_BATCH; ++k) {
            dot2_step(qb[k].x, pa[k].x, sb[k], cb[k]);
            dot2_step(qb[k].y, pa[k].y, sb[k], cb[k]);
            dot2_step(qb[k].z, pa[k].z, sb[k], cb[k]);
            dot2_step(qb[k].w, pa[k].w, sb[k], cb[k]);
          }
        }
      }
      auto finish = [&](const float (&s)[4], const float (&c)[4], int iv) {
        const ff lane_sum = ff_add(ff_add(ff_norm(s[0], c[0]), ff_norm(s[1], c[1])),
                                   ff_add(ff_norm(s[2], c[2]), ff_norm(s[3], c[3])));
        const ff v = ff_wave_sum(lane_sum.hi, lane_sum.lo);
        // (hi, lo) in lexicographic order, as ff_gt compares them
        if (lane == 0)
          atomicMax(&best_k[iv], ((unsigned long long)float_order(v.hi) << 32) | float_order(v.lo));
      };
      finish(sa, ca, i0);
      if (two) finish(sb, cb, i1);
    }
    __syncthreads();
    if (tid < mi) {
      const unsigned long long k = best_k[tid];
      // no masked view: 0
      mff_hi[tid] = k != 0ull ? order_float((uint32_t)(k >> 32)) : 0.f;
      mff_lo[tid] = k != 0ull ? order_float((uint32_t)k) : 0.f;
    }
    __syncthreads();
    if (tid == 0)
      for (int iv = 0; iv < mi; ++iv) acc = ff_add(acc, ff{mff_hi[iv], mff_lo[iv]});
  }
  if (tid == 0) {
    ff res = {0.f, 0.f};
    if (m > 0) res = ff_div_int(acc, m);
    s_hi[pair] = res.hi;
    s_lo[pair] = res.lo;
  }
}

size_t rescore_split_floats(int n_queries, int r) {
  const int64_t items = (int64_t)n_queries * ((r + RS_CANDS - 1) / RS_CANDS);
  if (items <= 0) return 0;
  return (size_t)min(items, RESCORE_SPLIT_ITEMS) * RESCORE_SPLIT * RS_CANDS * 64 * 64;
}

void launch_rescore(const float* master, int n_views, int dim,
                    const float* qviews, const int32_t* qoff, int n_queries,
                    int64_t ld, const int32_t* cand, int r, int top_k, float dot_err,
                    const int32_t* qwords, const int32_t* view_words, int ma,
                    const int32_t* active, const float* first_s, double first_err,
                    RescoreScratch sc, float* s_hi, float* s_lo, hipStream_t st) {
  const int64_t items = (int64_t)n_queries * ((r + RS_CANDS - 1) / RS_CANDS);
  if (items <= 0) return;
  // the storage bound as a float no smaller than it
  float fe = (float)first_err;
  if ((double)fe < first_err) fe = nextafterf(fe, INFINITY);
  const bool split = sc.part != nullptr && sc.n_split > 1;
  if (split) {
    // batches of at most RESCORE_SPLIT_ITEMS items (the kernels read the
    // batch size; the full kernel below takes the others)
    const int64_t si = min(items, RESCORE_SPLIT_ITEMS);
    hipLaunchKernelGGL(rescore_mask_kernel<RS_PART>, dim3((unsigned)(si * sc.n_split)),
                       dim3(RS_THREADS), 0, st, master, n_views, dim, qviews, qoff, n_queries,
                       cand, r, dot_err, qwords, view_words, ma, active, first_s, fe, top_k,
                       sc.mask, sc.s1, ld, sc.part, sc.n_split);
    hipLaunchKernelGGL(rescore_mask_kernel<RS_FINISH>, dim3((unsigned)si), dim3(RS_THREADS), 0,
                       st, master, n_views, dim, qviews, qoff, n_queries, cand, r, dot_err,
                       qwords, view_words, ma, active, first_s, fe, top_k, sc.mask, sc.s1, ld,
                       sc.part, sc.n_split);
  }
  if (!split || items > RESCORE_SPLIT_ITEMS)
    // grids cover every slot of the XCD-contiguous order
    hipLaunchKernelGGL(rescore_mask_kernel<RS_FULL>, dim3((unsigned)((items + 7) / 8 * 8)),
                       dim3(RS_THREADS), 0, st, master, n_views, dim, qviews, qoff, n_queries,
                       cand, r, dot_err, qwords, view_words, ma, active, first_s, fe, top_k,
                       sc.mask, sc.s1, ld, nullptr, split ? sc.n_split : 0);
  hipLaunchKernelGGL(rescore_mark_kernel, dim3((unsigned)n_queries), dim3(256), 0, st, sc.s1, ld,
                     qoff, r, top_k, dot_err, active, first_s, fe, sc.mark);
  const int64_t pairs = (int64_t)n_queries * r;
  hipLaunchKernelGGL(rescore_exact_kernel, dim3((unsigned)((pairs + 7) / 8 * 8)), dim3(256), 0, st,
                     master, n_views, dim, qviews, qoff, n_queries, cand, r, sc.mask, ld,
                     sc.mark, active, s_hi, s_lo);
}

// ------------------------------------------------------------------ final
struct Cand {
  float hi, lo;
  int32_t id;
};

__device__ inline bool cand_before(const Cand& a, const Cand& b) {
  if (a.hi != b.hi) return a.hi > b.hi;
  if (a.lo != b.lo) return a.lo > b.lo;
  return a.id < b.id;
}

__global__ __launch_bounds__(256) void final_rank_kernel(
    const int32_t* __restrict__ cand, const float* __restrict__ first_s,
    const float* __restrict__ s_hi, const float* __restrict__ s_lo, int r,
    int k, int64_t n_total, double first_err, const int32_t* __restrict__ qoff,
    const int32_t* __restrict__ overflow,
    const int32_t* __restrict__ active, int32_t* __restrict__ ids, float* __restrict__ scores,
    int32_t* __restrict__ flags) {
  __shared__ Cand c[MAX_R];
  const int b = blockIdx.x;
  if (active != nullptr && b >= *active) return;
  const int64_t base = (int64_t)b * r;
  int np2 = 1;
  while (np2 < r) np2 <<= 1;
  for (int i = threadIdx.x; i < np2; i += 256) {
    if (i < r) c[i] = Cand{s_hi[base + i], s_lo[base + i], cand[base + i]};
    else c[i] = Cand{-INFINITY, -INFINITY, 0x7fffffff};
  }
  __syncthreads();
  block_bitonic_sort(
      c, np2, [](const Cand& a, const Cand& b) { return cand_before(a, b); },
      [](const Cand& v, int j) {
        return Cand{__shfl_xor(v.hi, j, 64), __shfl_xor(v.lo, j, 64), __shfl_xor(v.id, j, 64)};
      });
  for (int i = threadIdx.x; i < k; i += 256) {
    ids[(int64_t)b * k + i] = c[i].id;
    scores[(int64_t)b * k + i] = c[i].hi;
  }
  if (flags != nullptr && threadIdx.x == 0) {
    // Any shape outside the candidates has a first-pass score at most the
    // smallest candidate's, so its exact score is below that plus the
    // first-pass error bound.  The list is complete when that stays below
    // the k-th exact score.
    bool complete = (int64_t)r >= n_total;
    if (!complete) {
      // the mean over this query's own views adds gamma_(m + 2)
      const double u = 5.9604644775390625e-08, nm = (double)(qoff[b + 1] - qoff[b]) + 2.0;
      const float err = (float)((first_err + nm * u / (1.0 - nm * u)) * 1.001);
      const float kth = c[k - 1].hi;
      const float bound = first_s[base + r - 1] + err;
      complete = bound < kth - fabsf(kth) * 2.4e-7f;
    }
    const bool ovf = overflow != nullptr && *overflow != 0;
    flags[b] = (complete && !ovf ? 1 : 0) | (ovf ? 2 : 0);
  }
}

void launch_final_rank(const int32_t* cand, const float* first_s,
                       const float* s_hi, const float* s_lo, int n_queries,
                       int r, int k, int64_t n_total, double first_err,
                       const int32_t* qoff, const int32_t* overflow, const int32_t* active,
                       int32_t* ids, float* scores, int32_t* flags, hipStream_t st) {
  if (n_queries <= 0) return;
  hipLaunchKernelGGL(final_rank_kernel, dim3(n_queries), dim3(256), 0, st,
                     cand, first_s, s_hi, s_lo, r, k, n_total, first_err, qoff, overflow,
                     active, ids, scores, flags);
}

}  // namespace gift
