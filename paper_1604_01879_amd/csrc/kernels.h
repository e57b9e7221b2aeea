// Host-side launchers of the GIFT kernels (internal interface).
#pragma once

#include "common.h"

namespace gift {

// Per-view scaled reduced-precision codes (BF16 or e4m3).
// scale: float32 per view (BF16 / FP8) or uint8 E8M0 per 32 values (MX).
void launch_quantize(const float* src, int64_t n, int dim, int dtype,
                     void* dst, void* scale, hipStream_t st);

// Eq. 3 first pass: for every database shape p and every query view c,
// mbuf[p * ldm + c] = max_j s(q_c, p_j) (scales applied for BF16/FP8).
// qv/qscale hold the query views in the same dtype as the database.
gift_status launch_score_tiles(const gift_views* db, const void* qv,
                               const void* qscale, int64_t total_q,
                               float* mbuf, int64_t ldm, hipStream_t st);

// Tile shape (0 or 1) per storage dtype and launch-order group of the
// first-pass scorer.
gift_status set_score_tuning(int dtype, int tile, int group);
void get_score_tuning(int dtype, int* tile, int* group);

// S[b][p] = (sum_{i in query b} mbuf[p][i]) / m_b.
void launch_reduce_queries(const float* mbuf, int64_t ldm, int64_t n_shapes,
                           const int32_t* qoff, int n_queries, float* S,
                           hipStream_t st);

// Top-r of each row of S [B][N] by (score desc, id asc), sorted.  In this
// and the next two launchers, rows (queries) b >= *active are skipped when
// `active` is not null (batch plans sized for more queries than a batch).
// tmp (select_top_ws bytes, may be 0) holds the chunk winners of long rows
// (null: one block per row).
size_t select_top_ws(int64_t n, int n_queries, int r);
void launch_select_top(const float* S, int64_t n, int n_queries, int r, const int32_t* active,
                       int32_t* out_id, float* out_s, void* tmp, hipStream_t st);

// Exact rescore of candidates: candidates whose first-pass score (first_s
// [queries][r], sorted desc) plus the first-pass bound first_err cannot
// reach the top_k are dropped first; then split-BF16 dot products with a
// known error bound give each view's candidate maxima and an approximate
// score; the candidates that can still reach the top_k get a compensated
// re-evaluation of every view pair that the bound cannot exclude as the
// maximum, and their float-float score; the others score -inf.
// With qwords != nullptr only pairs whose words match take part (Eq. 4).
struct RescoreScratch {
  unsigned long long* mask;  // [r][ld] view masks (candidate slot, query view)
  float* s1;                 // [r][ld] per-chunk sums of approximate maxima
  uint8_t* mark;             // [queries][r] candidates that can reach the top k
  // Split approximate phase (batches of at most RESCORE_SPLIT_ITEMS work
  // items whose queries have at most 64 views, decided per run from the
  // batch size): n_split blocks per work item each take a K range and
  // write their partial dot tiles to `part` (rescore_split_floats floats),
  // and a second kernel adds them in split order and builds the masks.
  // n_split 0: one block per item over the whole K range, always.
  float* part;
  int n_split;
};

// Floats of the split approximate phase's partial tiles for a capacity of
// n_queries x r candidates (work items of 4 candidates of one query; at
// most RESCORE_SPLIT_ITEMS of them are split).
size_t rescore_split_floats(int n_queries, int r);
constexpr int RESCORE_SPLIT = 4;            // K ranges per work item when split
constexpr int64_t RESCORE_SPLIT_ITEMS = 64;  // largest batch (in work items) that splits

// Rescore scratch from a workspace carver; ld = rows of query views the
// masks are indexed by (total or maximum views).
inline RescoreScratch take_rescore(Carver& c, int n_queries, int r, int64_t ld) {
  RescoreScratch s{};
  s.mask = c.take<unsigned long long>((size_t)r * ld);
  s.s1 = c.take<float>((size_t)r * ld);
  s.mark = c.take<uint8_t>((size_t)n_queries * r);
  return s;
}

void launch_rescore(const float* master, int n_views, int dim,
                    const float* qviews, const int32_t* qoff, int n_queries,
                    int64_t ld, const int32_t* cand, int r, int top_k, float dot_err,
                    const int32_t* qwords, const int32_t* view_words, int ma,
                    const int32_t* active, const float* first_s, double first_err,
                    RescoreScratch sc, float* s_hi, float* s_lo, hipStream_t st);

// Orders the r rescored candidates of each query by (exact score desc,
// id asc) and writes the top k; sets flags bit 0 when provably complete:
// the first-pass error bound of query b is first_err + gamma_(m_b + 2)
// (times 1.001), m_b = qoff[b + 1] - qoff[b] its view count.
// flags bit 1 is set when *overflow != 0 (a quantizer decision could not
// be certified); bit 0 then stays clear.
void launch_final_rank(const int32_t* cand, const float* first_s,
                       const float* s_hi, const float* s_lo, int n_queries,
                       int r, int k, int64_t n_total, double first_err,
                       const int32_t* qoff, const int32_t* overflow, const int32_t* active, int32_t* ids,
                       float* scores, int32_t* flags, hipStream_t st);

// ---- first inverted file
// words[r][a] = the a-th nearest codeword of row r (certified, ties to the
// lower index).  D holds chunk_rows x K floats; nhi/nlo K floats each;
// *overflow is incremented when a row has more than 256 candidates.
// xs (chunk_rows x dim x 4 bytes) and cbs (K x dim x 4 bytes): buffers for
// the BF16-split rows of the GEMM.
gift_status launch_assign(const float* x, int64_t n, int dim, const float* cb, int K, int ma,
                          int32_t* words, float* D, int64_t chunk_rows, float* nhi, float* nlo,
                          int32_t* overflow, uint8_t* xs, uint8_t* cbs, hipStream_t st);
size_t bucket_sort_ws(int64_t n, int K);
// Stable counting sort of items by key; off [K+1].  mode 0 writes item
// indices to out_a; mode 1 writes F-IF (shape, view) of item e = v*ma + a.
gift_status launch_bucket_sort(const int32_t* keys, int64_t n, int K, int64_t* off,
                               int mode, int ma, int n_views, int32_t* out_a, int32_t* out_b,
                               void* ws, hipStream_t st);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
void launch_gather_rows(const float* x, const int64_t* idx, int K, int dim, float* out,
                        hipStream_t st);
void launch_centroids(const float* x, int dim, int K, const int64_t* off, const int32_t* members,
                      const float* old_cb, float* new_cb, hipStream_t st);
void launch_count_changes(const int32_t* a, const int32_t* b, int64_t n, int32_t* cnt,
                          hipStream_t st);
gift_status launch_fif_scan(const gift_views* db, const int64_t* loff, const int32_t* ent_shape,
                            const int32_t* ent_view, int64_t n_entries, int K,
                            int64_t* tile_off, int64_t* tcount, const int64_t* goff,
                            const int32_t* gitems, const void* qv, const void* qscale,
                            uint32_t* mbuf, int64_t ldn, hipStream_t st);
// mbuf is [query view][shape] with row stride ldn (F-IF scan and reduce).
void launch_reduce_fif(const uint32_t* mbuf, int64_t ldn, int64_t n_shapes, const int32_t* qoff,
                       int n_queries, float* S, hipStream_t st);

// ---- persistent batch of the F-IF first pass
constexpr int BATCH_CTRL_WORDS = 8;
enum BatchPhase { BP_Q = 0, BP_GEMM, BP_FILL, BP_SEL, BP_PRE, BP_SCAT, BP_TILE, BP_SCAN, BP_RED,
                  BP_END };
constexpr int64_t BATCH_RED_SHAPES = 4096;            // shapes of one query per RED item
constexpr int64_t BATCH_Q_VIEWS = 4;                  // query views per Q item (one per wave)
// batches of at most this many views select each view's word with a whole
// block (one SEL item per view), larger ones with one wave per view
constexpr int64_t BATCH_SEL_SPLIT_MAX = 512;
struct BatchArgs {
  const uint8_t* db;
  const void* db_scale;      // per-view float32, E8M0 rows (MX) or null
  int n_views, row_bytes;
  int64_t n_shapes;
  const float* cb;
  const float* nhi;
  const float* nlo;
  int K, dim;
  const int64_t* loff;
  const int32_t* ent_shape;
  const int32_t* ent_view;
  const int64_t* tile_off;
  const int32_t* tile_word;  // list of each tile of the concatenated lists
  const float* qviews;
  uint8_t* qsplit;           // the batch's query views split into BF16 parts
  const uint8_t* cbsplit;    // the codebook split into BF16 parts
  int32_t* qoff;
  int Bmax;
  int64_t Vmax;
  const int32_t* desc;  // {n_queries, n_views} of the current batch
  uint8_t* qcodes;
  void* qscale;              // like db_scale, for the batch's query views
  float* D;
  int32_t* qwords;
  int32_t* counts;
  int64_t* goff;
  int32_t* fillc;
  int32_t* gitems;
  int32_t* act_off;          // [K] first active-tile slot of each word
  int32_t* act_tile;         // active list tiles of the batch
  uint32_t* mbuf;
  float* S;
  int32_t* overflow;
  unsigned long long* ctrl;  // [BATCH_CTRL_WORDS]: head, done, error, active tiles, Q done
  // [2 * BP_END + 1] wall-clock ticks: busy ticks per phase (waits
  // excluded), the last item end per phase, and the reset's start
  unsigned long long* phase_ticks;
  float gamma2;
  int64_t wait_ticks;        // wall-clock ticks a phase wait may take
  int64_t gemm_col_tiles;
  int tile_len;              // list entries per scan item (<= 128)
  int narrow_max;            // groups of at most this many views take the narrow tile
  // the split / quantize and codeword-dot work (and the match-buffer clear)
  // runs in launch_batch_pre's kernels before the persistent kernel, which
  // then has no Q or GEMM items
  int ext_gemm;
};
void launch_batch_reset(const BatchArgs& a, hipStream_t st);
// With ext_gemm: splits and codes the batch's query views and computes D
// (256 x 256 tiles, clearing the match buffer on the way) for the
// n_views = desc[1] rows of the current batch, grids sized for Vmax.
gift_status launch_batch_pre(const BatchArgs& a, int dtype, hipStream_t st);
gift_status launch_fif_batch(const BatchArgs& a, int dtype, int grid, hipStream_t st);
gift_status launch_norms(const float* cb, int K, int dim, float* nhi, float* nlo, hipStream_t st);
// n rows of dim float32 values split into BF16 parts, dim x 4 bytes per row:
// per 32 values, 32 high parts then 32 low parts (split_rows_kernel).
void launch_split_rows(const float* src, int64_t n, int dim, uint8_t* dst, hipStream_t st);
gift_status launch_list_tiles(const int64_t* loff, int K, int tile_len, int64_t* tcount,
                              int64_t* tile_off,
                              hipStream_t st);
void launch_tile_word(const int64_t* tile_off, int K, int32_t* tile_word, hipStream_t st);
float assign_gamma2(int dim);
// error bounds of the rescore dot product and of the first pass (api.hip)
float rescore_dot_error(int dim);
double first_pass_error(int dtype, int dim, bool list_scan);

// ---- second inverted file
// l1 [N][2] (compensated ||F_p||_1), post_off [N+1], post_id / post_val
// [<= N*k1]; cnt and fill are N-entry scratch counters.
void launch_build_sif(const int32_t* ids, const float* vals, int64_t N, int k1, float* l1,
                      int64_t* post_off, int32_t* post_id, float* post_val,
                      unsigned long long* cnt, unsigned long long* fill, hipStream_t st);
void launch_augment(const int32_t* t_ids, const float* t_val, int64_t N, int k1,
                    const int32_t* members, int k2, const int32_t* own_ids, const float* own_val,
                    int k_own, int n_rows, int32_t* out_ids, float* out_val, int k_out,
                    int32_t* n_members, hipStream_t st);
void launch_fuse_self(const float* self1, const int32_t* n1, const float* self2,
                      const int32_t* n2, float alpha, int n_rows, float* out, hipStream_t st);
void launch_fuse(const int32_t* i1, const float* v1, int k_a, const int32_t* i2, const float* v2,
                 int k_b, float alpha, int n_rows, int32_t* out_ids, float* out_val, int k_out,
                 hipStream_t st);
void launch_rerank_sif(const float* l1, const int64_t* post_off, const int32_t* post_id,
                       const float* post_val, int64_t N, const int32_t* q_id, const float* q_val,
                       const float* q_self, int B, int k1, int k, int32_t* out_id, float* out_s,
                       int32_t* flags, hipStream_t st);

}  // namespace gift
