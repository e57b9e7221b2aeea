// The second inverted file (Sec. 2.4): sparse activations F (Eq. 7), their
// L1 norms, the postings of Fig. 3, and re-ranking by the fuzzy Jaccard
// similarity of Eq. 8 evaluated through Eq. 13 (numerator over shared
// non-zero coordinates) and Eq. 14 (denominator from the L1 norms).
#include "bitonic.h"
#include "kernels.h"

namespace gift {

// ------------------------------------------------------------------ build
// ||F_p||_1 as a compensated sum of the memberships in rank order, and the
// per-coordinate posting counts.  Valid entries: id in [0, N), value > 0.
__global__ __launch_bounds__(256) void sif_count_kernel(const int32_t* __restrict__ ids,
                                                        const float* __restrict__ vals,
                                                        int64_t N, int k1,
                                                        float* __restrict__ l1,
                                                        unsigned long long* __restrict__ cnt) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  ff acc = {0.f, 0.f};
  for (int r = 0; r < k1; ++r) {
    const int32_t i = ids[p * k1 + r];
    if (i < 0 || i >= N) continue;
    const float v = vals[p * k1 + r];
    acc = ff_add(acc, ff{v, 0.f});
    if (v > 0.f) atomicAdd(&cnt[i], 1ull);
  }
  l1[2 * p] = acc.hi;
  l1[2 * p + 1] = acc.lo;
}

__global__ __launch_bounds__(256) void sif_scatter_kernel(const int32_t* __restrict__ ids,
                                                          const float* __restrict__ vals,
                                                          int64_t N, int k1,
                                                          const int64_t* __restrict__ off,
                                                          unsigned long long* __restrict__ fill,
                                                          int32_t* __restrict__ post_id,
                                                          float* __restrict__ post_val) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= N * k1) return;
  const int32_t i = ids[e];
  const float v = vals[e];
  if (i < 0 || i >= N || !(v > 0.f)) return;
  const int64_t pos = off[i] + (int64_t)atomicAdd(&fill[i], 1ull);
  post_id[pos] = (int32_t)(e / k1);
  post_val[pos] = v;
}

// Orders each posting list by shape id (lists are short: insertion sort).
__global__ __launch_bounds__(256) void sif_sort_kernel(const int64_t* __restrict__ off, int64_t N,
                                                       int32_t* __restrict__ post_id,
                                                       float* __restrict__ post_val) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int64_t a = off[i], b = off[i + 1];
  for (int64_t x = a + 1; x < b; ++x) {
    const int32_t pid = post_id[x];
    const float pv = post_val[x];
    int64_t y = x - 1;
    while (y >= a && post_id[y] > pid) {
      post_id[y + 1] = post_id[y];
      post_val[y + 1] = post_val[y];
      --y;
    }
    post_id[y + 1] = pid;
    post_val[y + 1] = pv;
  }
}

// The count array doubles as int64 input of the exclusive scan.
__global__ __launch_bounds__(1024) void scan_counts_kernel(const unsigned long long* __restrict__ cnt,
                                                           int64_t K, int64_t* __restrict__ off) {
  __shared__ int64_t part[1024];
  const int64_t per = (K + 1023) / 1024;
  const int64_t k0 = threadIdx.x * per;
  int64_t s = 0;
  for (int64_t k = k0; k < k0 + per && k < K; ++k) s += (int64_t)cnt[k];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - s;
  for (int64_t k = k0; k < k0 + per && k < K; ++k) {
    off[k] = run;
    run += (int64_t)cnt[k];
  }
  if (threadIdx.x == 1023) off[K] = part[1023];
}

__global__ void zero_u64_kernel(unsigned long long* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0ull;
}

void launch_build_sif(const int32_t* ids, const float* vals, int64_t N, int k1, float* l1,
                      int64_t* post_off, int32_t* post_id, float* post_val,
                      unsigned long long* cnt, unsigned long long* fill, hipStream_t st) {
  const int64_t zb = (N + 255) / 256 < 65536 ? (N + 255) / 256 : 65536;
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)zb), dim3(256), 0, st, cnt, N);
  hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)zb), dim3(256), 0, st, fill, N);
  hipLaunchKernelGGL(sif_count_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, ids,
                     vals, N, k1, l1, cnt);
  hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(1024), 0, st, cnt, N, post_off);
  hipLaunchKernelGGL(sif_scatter_kernel, dim3((unsigned)((N * k1 + 255) / 256)), dim3(256), 0,
                     st, ids, vals, N, k1, post_off, fill, post_id, post_val);
  hipLaunchKernelGGL(sif_sort_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                     post_off, N, post_id, post_val);
}

// ------------------------------------------------------------------ rerank
// One block per query.  F_q has memberships q_val at coordinates q_id (ids
// < 0 skipped) plus q_self for the query itself, which has no coordinate and
// only enters ||F_q||_1.  The postings of the query's coordinates are
// expanded into LDS as (shape, min(F_q[i], F_p[i])) pairs, sorted by
// (shape, expansion order); each shape's pairs are summed (Eq. 13), the
// score S' = num / (||F_q||_1 + ||F_p||_1 - num) (Eq. 14) is formed in
// compensated arithmetic, and the shapes are ranked by (S' desc, id asc);
// shapes sharing no coordinate score 0 and fill the list in id order.
//
// Every posting list is sorted by shape, so the postings of the shapes
// below a bound p_hi form a prefix of each list.  When a query's postings
// exceed SIF_CAP, the block walks the shape axis in passes: each pass takes
// the largest p_hi whose prefixes fit SIF_CAP (a shape has at most k1 <=
// 256 postings, so every pass advances), scores those shapes exactly as a
// single pass would (a shape's postings all fall in one pass, in the same
// order), and merges its best shapes into the running top k.  The result is
// the same for any posting count.
constexpr int SIF_CAP = 4096;      // expanded postings per pass
constexpr int SIF_KMAX = 1024;     // largest top_k
constexpr int SIF_THREADS = 1024;  // one block per query; its LDS leaves room for one per CU
constexpr int SIF_WAVES = SIF_THREADS / 64;

struct SCand {
  float hi, lo;
  int32_t id;
};

__device__ inline bool scand_before(const SCand& a, const SCand& b) {
  if (a.hi != b.hi) return a.hi > b.hi;
  if (a.lo != b.lo) return a.lo > b.lo;
  return a.id < b.id;
}

// (a.hi + a.lo) / (b.hi + b.lo) for b > 0.
__device__ inline ff ff_div(ff a, ff b) {
#pragma clang fp contract(off)
  const float q1 = a.hi / b.hi;
  float p, e;
  two_prod(q1, b.hi, p, e);
  // remainder a - q1 * b
  float r = ((a.hi - p) - e) + a.lo;
  r = r - q1 * b.lo;
  const float q2 = r / b.hi;
  return ff_norm(q1, q2);
}

// Sum (op 0) or minimum (op 1) of v over the block; every thread gets it.
__device__ inline int64_t sif_block_reduce(int64_t v, int op, int64_t* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t w = __shfl_xor(v, o, 64);
    v = op == 0 ? v + w : (w < v ? w : v);
  }
  if (lane == 0) red[wave] = v;
  __syncthreads();
  int64_t t = red[0];
  for (int w = 1; w < SIF_WAVES; ++w) t = op == 0 ? t + red[w] : (red[w] < t ? red[w] : t);
  __syncthreads();
  return t;
}

// First position in [lo, hi) of the ascending ids whose id is >= x.
__device__ inline int64_t sif_lower_bound(const int32_t* __restrict__ ids, int64_t lo, int64_t hi,
                                          int64_t x) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)ids[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(SIF_THREADS) void rerank_sif_kernel(
    const float* __restrict__ l1, const int64_t* __restrict__ post_off,
    const int32_t* __restrict__ post_id, const float* __restrict__ post_val, int64_t N,
    const int32_t* __restrict__ q_id, const float* __restrict__ q_val,
    const float* __restrict__ q_self, int k1, int k, int32_t* __restrict__ out_id,
    float* __restrict__ out_s, int32_t* __restrict__ flags) {
  __shared__ int64_t pre[257];
  __shared__ int64_t cur_r[256];   // next unused posting of coordinate r
  __shared__ int64_t end_r[256];   // end of coordinate r's postings
  __shared__ int64_t take_r[256];  // postings of coordinate r in this pass
  __shared__ float val_r[256];     // membership at coordinate r
  __shared__ uint8_t in_r[256];    // coordinate r names a shape in range
  __shared__ int64_t red[SIF_WAVES];
  __shared__ float Ahi, Alo;
  __shared__ int wsum[SIF_WAVES];
  __shared__ int n_best;
  extern __shared__ __align__(16) uint8_t sm[];
  uint64_t* key = reinterpret_cast<uint64_t*>(sm);                // (shape << 32) | slot
  float* pv = reinterpret_cast<float*>(sm + 8 * SIF_CAP);           // min value per slot
  SCand* cand = reinterpret_cast<SCand*>(sm + 12 * SIF_CAP);        // this pass's shapes
  SCand* best = cand + SIF_CAP;                                     // running top k
  SCand* best2 = best + SIF_KMAX;                                   // merge output
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int32_t* qi = q_id + (int64_t)b * k1;
  const float* qv = q_val + (int64_t)b * k1;

  // the coordinates' posting ranges, loaded in parallel; then ||F_q||_1 in
  // coordinate order
  for (int r = tid; r < k1; r += SIF_THREADS) {
    const int32_t i = qi[r];
    const bool ok = i >= 0 && i < N;
    const float v = qv[r];
    const bool use = ok && v > 0.f;
    cur_r[r] = use ? post_off[i] : 0;
    end_r[r] = use ? post_off[i + 1] : 0;
    val_r[r] = v;
    in_r[r] = ok;
  }
  __syncthreads();
  if (tid == 0) {
    ff A = {q_self != nullptr ? q_self[b] : 0.f, 0.f};
    for (int r = 0; r < k1; ++r)
      if (in_r[r]) A = ff_add(A, ff{val_r[r], 0.f});
    Ahi = A.hi;
    Alo = A.lo;
    n_best = 0;
  }
  __syncthreads();
  int passes = 0;
  for (;;) {
    // postings left, over the coordinates
    const int64_t left =
        sif_block_reduce(tid < k1 ? end_r[tid] - cur_r[tid] : 0, 0, red);
    if (left == 0) break;
    ++passes;
    if (left <= SIF_CAP) {
      if (tid < k1) take_r[tid] = end_r[tid] - cur_r[tid];
    } else {
      // largest p_hi with at most SIF_CAP postings of shapes below it:
      // count(lo) <= SIF_CAP < count(hi), lo starting just past the smallest
      // shape left (at most k1 postings) and hi above every int32 id (all
      // postings); each pass takes at least the smallest shape's postings
      const int64_t pmin = sif_block_reduce(
          tid < k1 && cur_r[tid] < end_r[tid] ? (int64_t)post_id[cur_r[tid]] : ((int64_t)1 << 31),
          1, red);
      int64_t lo = pmin + 1, hi = (int64_t)1 << 31;
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        const int64_t c = sif_block_reduce(
            tid < k1 ? sif_lower_bound(post_id, cur_r[tid], end_r[tid], mid) - cur_r[tid] : 0, 0,
            red);
        if (c <= SIF_CAP) lo = mid; else hi = mid;
      }
      if (tid < k1) take_r[tid] = sif_lower_bound(post_id, cur_r[tid], end_r[tid], lo) - cur_r[tid];
    }
    __syncthreads();
    if (tid == 0) {
      int64_t run = 0;
      for (int r = 0; r < k1; ++r) {
        pre[r] = run;
        run += take_r[r];
      }
      pre[k1] = run;
    }
    __syncthreads();
    const int L = (int)pre[k1];  // <= SIF_CAP
    for (int s = tid; s < L; s += SIF_THREADS) {
      int lo = 0, hi = k1;  // r with pre[r] <= s < pre[r+1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= s) lo = mid; else hi = mid;
      }
      const int64_t e = cur_r[lo] + (s - pre[lo]);
      key[s] = ((uint64_t)(uint32_t)post_id[e] << 32) | (uint32_t)s;
      pv[s] = fminf(val_r[lo], post_val[e]);
    }
    int np2 = 1;
    while (np2 < L) np2 <<= 1;
    for (int s = L + tid; s < np2; s += SIF_THREADS) key[s] = ~0ull;
    __syncthreads();
    block_bitonic_sort(
        key, np2, [](uint64_t a, uint64_t b) { return a < b; },
        [](uint64_t v, int j) { return (uint64_t)__shfl_xor((unsigned long long)v, j, 64); });
    // one candidate per distinct shape, in ascending shape order
    int base_u = 0;
    for (int s0 = 0; s0 < L; s0 += SIF_THREADS) {
      const int s = s0 + tid;
      const bool start = s < L && (s == 0 || (key[s] >> 32) != (key[s - 1] >> 32));
      const int lane = tid & 63, wave = tid >> 6;
      const unsigned long long bal = __ballot(start);
      if (lane == 0) wsum[wave] = __popcll(bal);
      __syncthreads();
      int before = 0, tot = 0;
      for (int w = 0; w < SIF_WAVES; ++w) {
        if (w < wave) before += wsum[w];
        tot += wsum[w];
      }
      const int u = base_u + before + __popcll(bal & ((1ull << lane) - 1ull));
      if (start) {
        const int32_t p = (int32_t)(key[s] >> 32);
        ff num = {0.f, 0.f};
        for (int t = s; t < L && (key[t] >> 32) == (uint64_t)(uint32_t)p; ++t)
          num = ff_add(num, ff{pv[(uint32_t)key[t]], 0.f});
        // denominator ||F_q||_1 + ||F_p||_1 - num (Eq. 14)
        ff den = ff_add(ff{Ahi, Alo}, ff{l1[2 * (int64_t)p], l1[2 * (int64_t)p + 1]});
        den = ff_add(den, ff{-num.hi, -num.lo});
        const ff sc = ff_div(num, den);
        cand[u] = SCand{sc.hi, sc.lo, p};
      }
      base_u += tot;
      __syncthreads();
    }
    const int U = base_u;
    int np2u = 1;
    while (np2u < U) np2u <<= 1;
    for (int i = U + tid; i < np2u; i += SIF_THREADS) cand[i] = SCand{-INFINITY, -INFINITY, 0x7fffffff};
    __syncthreads();
    block_bitonic_sort(
        cand, np2u, [](const SCand& a, const SCand& b) { return scand_before(a, b); },
        [](const SCand& v, int j) {
          return SCand{__shfl_xor(v.hi, j, 64), __shfl_xor(v.lo, j, 64), __shfl_xor(v.id, j, 64)};
        });
    // merge the pass's best min(U, k) into the running top k: an element's
    // output rank is its rank in its own list plus the number of elements of
    // the other list ordered before it (shapes of different passes differ)
    const int nA = U < k ? U : k, nB = n_best;
    for (int i = tid; i < nA; i += SIF_THREADS) {
      const SCand x = cand[i];
      int lo = 0, hi = nB;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (scand_before(best[mid], x)) lo = mid + 1; else hi = mid;
      }
      if (i + lo < k) best2[i + lo] = x;
    }
    for (int j = tid; j < nB; j += SIF_THREADS) {
      const SCand y = best[j];
      int lo = 0, hi = nA;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (scand_before(cand[mid], y)) lo = mid + 1; else hi = mid;
      }
      if (j + lo < k) best2[j + lo] = y;
    }
    __syncthreads();
    const int nn = nA + nB < k ? nA + nB : k;
    for (int i = tid; i < nn; i += SIF_THREADS) best[i] = best2[i];
    if (tid < k1) cur_r[tid] += take_r[tid];
    if (tid == 0) n_best = nn;
    __syncthreads();
  }
  const int kp = n_best;
  for (int i = tid; i < kp; i += SIF_THREADS) {
    out_id[(int64_t)b * k + i] = best[i].id;
    out_s[(int64_t)b * k + i] = best[i].hi;
  }
  if (kp < k) {
    // every shape with a shared coordinate is in `best`: sort its ids to
    // skip them in the zero-score padding
    int np2k = 1;
    while (np2k < kp) np2k <<= 1;
    for (int i = tid; i < np2k; i += SIF_THREADS)
      key[i] = i < kp ? (uint64_t)(uint32_t)best[i].id : ~0ull;
    __syncthreads();
    block_bitonic_sort(
        key, np2k, [](uint64_t a, uint64_t b) { return a < b; },
        [](uint64_t v, int j) { return (uint64_t)__shfl_xor((unsigned long long)v, j, 64); });
    if (tid == 0) {
      // zero-score shapes in id order, skipping the candidates
      int pos = kp, c = 0;
      for (int64_t id = 0; pos < k && id < N; ++id) {
        while (c < kp && (int64_t)key[c] < id) ++c;
        if (c < kp && (int64_t)key[c] == id) continue;
        out_id[(int64_t)b * k + pos] = (int32_t)id;
        out_s[(int64_t)b * k + pos] = 0.f;
        ++pos;
      }
    }
  }
  if (tid == 0 && flags != nullptr) flags[b] = passes > 1 ? 3 : 1;
}

// ------------------------------------------------------------------ augment
// Neighbour augmentation (Eq. 10): output row b is the mean of its member
// rows, F_b := (1/n) sum over the valid members i of F_i, where member j of
// row b is table row members[b][j] (ids < 0 skipped) and, when own_ids is
// given, the row's own list counts as one more member.  One block per row:
// the (id, value) pairs of all members are gathered into LDS, sorted by
// (id, member), summed per id in that order and divided by n; the result is
// written in ascending id, padded with (-1, 0).
constexpr int AUG_CAP = 1024;

__global__ __launch_bounds__(256) void augment_kernel(
    const int32_t* __restrict__ t_ids, const float* __restrict__ t_val, int64_t N, int k1,
    const int32_t* __restrict__ members, int k2, const int32_t* __restrict__ own_ids,
    const float* __restrict__ own_val, int k_own, int32_t* __restrict__ out_ids,
    float* __restrict__ out_val, int k_out, int32_t* __restrict__ n_members) {
  __shared__ uint64_t key[AUG_CAP];  // (id << 32) | slot
  __shared__ float val[AUG_CAP];
  __shared__ int nmem;
  const int b = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) {
    int n = own_ids != nullptr ? 1 : 0;
    for (int j = 0; j < k2; ++j) {
      const int32_t m = members[(int64_t)b * k2 + j];
      if (m >= 0 && m < N) ++n;
    }
    nmem = n;
  }
  __syncthreads();
  // slot order: members in order, then the own row
  const int total = k2 * k1 + (own_ids != nullptr ? k_own : 0);
  for (int s = tid; s < total; s += 256) {
    int32_t id = -1;
    float v = 0.f;
    if (s < k2 * k1) {
      const int32_t m = members[(int64_t)b * k2 + s / k1];
      if (m >= 0 && m < N) {
        id = t_ids[(int64_t)m * k1 + s % k1];
        v = t_val[(int64_t)m * k1 + s % k1];
      }
    } else {
      id = own_ids[(int64_t)b * k_own + (s - k2 * k1)];
      v = own_val[(int64_t)b * k_own + (s - k2 * k1)];
    }
    key[s] = (id >= 0 && id < N) ? (((uint64_t)(uint32_t)id << 32) | (uint32_t)s) : ~0ull;
    val[s] = v;
  }
  int np2 = 1;
  while (np2 < total) np2 <<= 1;
  for (int s = total + tid; s < np2; s += 256) key[s] = ~0ull;
  __syncthreads();
  for (int kk = 2; kk <= np2; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < np2; i += 256) {
        const int ix = i ^ j;
        if (ix > i) {
          const bool up = (i & kk) == 0;
          const uint64_t x = key[i], y = key[ix];
          if ((x > y) == up) { key[i] = y; key[ix] = x; }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    const float nf = nmem > 0 ? (float)nmem : 1.f;
    int o = 0;
    for (int s = 0; s < total && key[s] != ~0ull;) {
      const uint32_t id = (uint32_t)(key[s] >> 32);
      float sum = 0.f;
      int t = s;
      for (; t < total && key[t] != ~0ull && (uint32_t)(key[t] >> 32) == id; ++t)
        sum += val[(uint32_t)key[t]];
      if (o < k_out) {
        out_ids[(int64_t)b * k_out + o] = (int32_t)id;
        out_val[(int64_t)b * k_out + o] = sum / nf;
      }
      ++o;
      s = t;
    }
    for (; o < k_out; ++o) {
      out_ids[(int64_t)b * k_out + o] = -1;
      out_val[(int64_t)b * k_out + o] = 0.f;
    }
    if (n_members != nullptr) n_members[b] = nmem;
  }
}

void launch_augment(const int32_t* t_ids, const float* t_val, int64_t N, int k1,
                    const int32_t* members, int k2, const int32_t* own_ids, const float* own_val,
                    int k_own, int n_rows, int32_t* out_ids, float* out_val, int k_out,
                    int32_t* n_members, hipStream_t st) {
  if (n_rows <= 0) return;
  hipLaunchKernelGGL(augment_kernel, dim3(n_rows), dim3(256), 0, st, t_ids, t_val, N, k1,
                     members, k2, own_ids, own_val, k_own, out_ids, out_val, k_out, n_members);
}

// ------------------------------------------------------------------ fusion
// Eq. 9: aggregated contextual activation of two measures, the element-wise
// generalised mean ((F1^a + F2^a) / 2)^(1/a) over the union of the two
// rows' coordinates (a coordinate missing from one row has membership 0
// there).  One block per row; ids are distinct within a row.
__global__ __launch_bounds__(256) void fuse_kernel(
    const int32_t* __restrict__ i1, const float* __restrict__ v1, int k_a,
    const int32_t* __restrict__ i2, const float* __restrict__ v2, int k_b, float alpha,
    int32_t* __restrict__ out_ids, float* __restrict__ out_val, int k_out) {
  __shared__ uint64_t key[AUG_CAP];  // (id << 32) | slot
  __shared__ float val[AUG_CAP];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int total = k_a + k_b;
  for (int s = tid; s < total; s += 256) {
    const int32_t id = s < k_a ? i1[(int64_t)b * k_a + s] : i2[(int64_t)b * k_b + (s - k_a)];
    const float v = s < k_a ? v1[(int64_t)b * k_a + s] : v2[(int64_t)b * k_b + (s - k_a)];
    key[s] = id >= 0 ? (((uint64_t)(uint32_t)id << 32) | (uint32_t)s) : ~0ull;
    val[s] = v;
  }
  int np2 = 1;
  while (np2 < total) np2 <<= 1;
  for (int s = total + tid; s < np2; s += 256) key[s] = ~0ull;
  __syncthreads();
  for (int kk = 2; kk <= np2; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < np2; i += 256) {
        const int ix = i ^ j;
        if (ix > i) {
          const bool up = (i & kk) == 0;
          const uint64_t x = key[i], y = key[ix];
          if ((x > y) == up) { key[i] = y; key[ix] = x; }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    const float inv_a = 1.f / alpha;
    int o = 0;
    for (int s = 0; s < total && key[s] != ~0ull;) {
      const uint32_t id = (uint32_t)(key[s] >> 32);
      float a = 0.f, c = 0.f;
      int t = s;
      for (; t < total && key[t] != ~0ull && (uint32_t)(key[t] >> 32) == id; ++t) {
        const uint32_t slot = (uint32_t)key[t];
        if ((int)slot < k_a) a = val[slot]; else c = val[slot];
      }
      const float pa = a > 0.f ? powf(a, alpha) : 0.f;
      const float pc = c > 0.f ? powf(c, alpha) : 0.f;
      const float m = 0.5f * (pa + pc);
      if (o < k_out) {
        out_ids[(int64_t)b * k_out + o] = (int32_t)id;
        out_val[(int64_t)b * k_out + o] = m > 0.f ? powf(m, inv_a) : 0.f;
      }
      ++o;
      s = t;
    }
    for (; o < k_out; ++o) {
      out_ids[(int64_t)b * k_out + o] = -1;
      out_val[(int64_t)b * k_out + o] = 0.f;
    }
  }
}

// Self membership of outside queries through Eq. 11 then Eq. 9: under each
// measure the query's own membership self / n after averaging over its n
// members, then the generalised mean of the two with the fuse kernel's
// arithmetic.
__global__ __launch_bounds__(256) void fuse_self_kernel(const float* __restrict__ self1,
                                                        const int32_t* __restrict__ n1,
                                                        const float* __restrict__ self2,
                                                        const int32_t* __restrict__ n2,
                                                        float alpha, int n_rows,
                                                        float* __restrict__ out) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= n_rows) return;
  const float inv_a = 1.f / alpha;
  const float a = n1[b] > 0 ? self1[b] / (float)n1[b] : 0.f;
  const float c = n2[b] > 0 ? self2[b] / (float)n2[b] : 0.f;
  const float pa = a > 0.f ? powf(a, alpha) : 0.f;
  const float pc = c > 0.f ? powf(c, alpha) : 0.f;
  const float m = 0.5f * (pa + pc);
  out[b] = m > 0.f ? powf(m, inv_a) : 0.f;
}

void launch_fuse_self(const float* self1, const int32_t* n1, const float* self2,
                      const int32_t* n2, float alpha, int n_rows, float* out, hipStream_t st) {
  if (n_rows <= 0) return;
  hipLaunchKernelGGL(fuse_self_kernel, dim3((n_rows + 255) / 256), dim3(256), 0, st, self1, n1,
                     self2, n2, alpha, n_rows, out);
}

void launch_fuse(const int32_t* i1, const float* v1, int k_a, const int32_t* i2, const float* v2,
                 int k_b, float alpha, int n_rows, int32_t* out_ids, float* out_val, int k_out,
                 hipStream_t st) {
  if (n_rows <= 0) return;
  hipLaunchKernelGGL(fuse_kernel, dim3(n_rows), dim3(256), 0, st, i1, v1, k_a, i2, v2, k_b,
                     alpha, out_ids, out_val, k_out);
}

void launch_rerank_sif(const float* l1, const int64_t* post_off, const int32_t* post_id,
                       const float* post_val, int64_t N, const int32_t* q_id, const float* q_val,
                       const float* q_self, int B, int k1, int k, int32_t* out_id, float* out_s,
                       int32_t* flags, hipStream_t st) {
  if (B <= 0) return;
  const size_t shmem = (size_t)SIF_CAP * (8 + 4 + sizeof(SCand)) + 2 * (size_t)SIF_KMAX * sizeof(SCand);
  (void)ensure_dynamic_lds(reinterpret_cast<const void*>(rerank_sif_kernel), shmem);
  hipLaunchKernelGGL(rerank_sif_kernel, dim3(B), dim3(SIF_THREADS), shmem, st, l1, post_off, post_id,
                     post_val, N, q_id, q_val, q_self, k1, k, out_id, out_s, flags);
}

}  // namespace gift
