// Host-side launchers of the GIFT kernels (internal interface).
#pragma once

#include "common.h"

namespace gift {

// Per-view scaled reduced-precision codes (BF16 or e4m3).
void launch_quantize(const float* src, int64_t n, int dim, int dtype,
                     void* dst, float* scale, hipStream_t st);

// Eq. 3 first pass: for every database shape p and every query view c,
// mbuf[p * ldm + c] = max_j s(q_c, p_j) (scales applied for BF16/FP8).
// qv/qscale hold the query views in the same dtype as the database.
gift_status launch_score_tiles(const gift_views* db, const void* qv,
                               const float* qscale, int64_t total_q,
                               float* mbuf, int64_t ldm, hipStream_t st);

// S[b][p] = (sum_{i in query b} mbuf[p][i]) / m_b.
void launch_reduce_queries(const float* mbuf, int64_t ldm, int64_t n_shapes,
                           const int32_t* qoff, int n_queries, float* S,
                           hipStream_t st);

// Top-r of each row of S [B][N] by (score desc, id asc), sorted.
void launch_select_top(const float* S, int64_t n, int n_queries, int r,
                       int32_t* out_id, float* out_s, hipStream_t st);

// Exact rescore of candidates: float32 dot products with a known error
// bound, then a compensated re-evaluation of every view pair that float32
// rounding could make the maximum.  Writes the float-float score.
void launch_rescore(const float* master, int n_views, int dim,
                    const float* qviews, const int32_t* qoff, int n_queries,
                    int max_m, const int32_t* cand, int r, float dot_err,
                    float* s_hi, float* s_lo, hipStream_t st);

// Orders the r rescored candidates of each query by (exact score desc,
// id asc) and writes the top k; sets flags bit 0 when provably complete.
void launch_final_rank(const int32_t* cand, const float* first_s,
                       const float* s_hi, const float* s_lo, int n_queries,
                       int r, int k, int64_t n_total, float first_err,
                       int32_t* ids, float* scores, int32_t* flags,
                       hipStream_t st);

}  // namespace gift
