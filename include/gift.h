/*
 * gift.h -- C ABI of the GIFT search-stage library for AMD MI355X (gfx950).
 *
 * The calls follow the paper's statement of the search problem
 * (Bai et al., "GIFT: A Real-time and Scalable 3D Shape Search Engine",
 * arXiv 1604.01879, Sec. 2.3 and 2.4):
 *
 *   a database X = {x_1..x_N} of shapes, each a set V(x) of N_v view
 *   features; a query x_q with its own view set; the multi-view matching
 *   function S of Eq. 3; its inverted-file approximation of Eq. 4 with a
 *   k-means vocabulary B = {b_1..b_K} and quantizer c(x); and the
 *   contextual re-ranking S' of Eq. 8 evaluated through the second
 *   inverted file (Eq. 13, 14).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers are DEVICE pointers owned by the caller unless the argument
 *    comment says "host".  The library never allocates device memory:
 *    every call that needs scratch space takes a caller-owned workspace
 *    (ws, ws_bytes) whose minimum size the matching *_workspace() function
 *    returns.  Workspace contents need not be initialised.
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL is the default stream) unless it says it synchronises.
 *  - Every call returns a gift_status.  On failure, gift_last_error()
 *    returns a message for the calling thread.  Nothing throws across the
 *    ABI.  No pointer is retained after a call returns.
 *  - Views are float32 rows of `dim` values, shape-major: database view j
 *    of shape p is row p * n_views + j.  dim must be a multiple of 32.
 *    Arrays of rows (views, master views, query views, codebooks, training
 *    rows) must be 16-byte aligned and scale arrays 4-byte aligned;
 *    otherwise a call returns GIFT_EINVAL.
 *    The paper's features are L2-normalised (Sec. 2.2); the certified
 *    ranking below assumes unit-norm rows (to within 1e-6).
 *  - Discrete outputs (codeword assignments, ranked ids) are defined on the
 *    exact value of the quantity over the float32 inputs.  The kernels
 *    compute in float32 and settle every decision that float32 rounding
 *    could flip with a compensated (float-float) re-evaluation, so the
 *    result equals the exact decision; equal exact values go to the lower
 *    index.  Scores are returned as float32.
 */
#ifndef GIFT_H
#define GIFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gift_status;
#define GIFT_OK            0
#define GIFT_EINVAL       (-1)  /* bad argument (null pointer, size, range) */
#define GIFT_EWORKSPACE   (-2)  /* workspace smaller than *_workspace()      */
#define GIFT_EUNSUPPORTED (-3)  /* dtype, device arch or dim not supported   */
#define GIFT_EHIP         (-4)  /* a HIP runtime call failed                 */
#define GIFT_ECAPACITY    (-5)  /* an output or index capacity was exceeded  */

/* Storage formats of database views. */
#define GIFT_F32      0   /* float32                                          */
#define GIFT_BF16     1   /* bfloat16 code, value = code * scale[view]         */
#define GIFT_FP8E4M3  2   /* OCP e4m3fn code (max 448), value = code * scale   */
#define GIFT_MXFP8    3   /* e4m3 codes, one E8M0 scale byte per 32 values     */
#define GIFT_MXFP4    4   /* e2m1 codes (two per byte, even index in the low
                             nibble), one E8M0 scale byte per 32 values       */

/* Database views (Sec. 2.3: V(x_p) = {p_1..p_Nv}). */
typedef struct gift_views {
  const void*  data;      /* [n_shapes * n_views][dim] codes of `dtype`       */
  int32_t      dtype;     /* GIFT_F32 / GIFT_BF16 / GIFT_FP8E4M3              */
  int32_t      n_views;   /* N_v, 1..64                                       */
  int64_t      n_shapes;  /* N                                                */
  int32_t      dim;       /* d, multiple of 32                                */
  int32_t      _pad;
  const void*  scale;     /* BF16 / FP8: float32 per view [n_shapes*n_views];
                             MX: uint8 E8M0 [n_shapes*n_views][dim/32], the
                             value of a code is code * 2^(e8m0 - 127);
                             NULL for F32                                     */
  const float* master;    /* float32 copy [n_shapes * n_views][dim]; required
                             for the float32 rescore when dtype != GIFT_F32;
                             may equal `data` when dtype == GIFT_F32          */
} gift_views;

/* A batch of query shapes with ragged view counts (V(x_q)). */
typedef struct gift_queries {
  const float*   views;       /* [total_views][dim] float32                   */
  const int32_t* offsets;     /* [n_queries + 1] device, offsets[0] = 0        */
  int32_t        n_queries;   /* B                                            */
  int32_t        max_views;   /* host bound: max_b (offsets[b+1]-offsets[b]) */
  int64_t        total_views; /* host: offsets[n_queries]                      */
} gift_queries;

const char* gift_version(void);
const char* gift_last_error(void);

/* ---------------------------------------------------------------------- */
/* Reduced-precision storage of view features.                            */
/* BF16 / FP8: scale[v] = max_t |src[v][t]| / Fmax (Fmax = 1 for BF16, 448 */
/* for e4m3), dst[v][t] = round_nearest_even_saturating(src[v][t] /        */
/* scale[v]); an all-zero row gets scale 1.  dst is [n][dim] of 2-byte     */
/* (BF16) or 1-byte (e4m3) codes; `scale` is float32 [n].                  */
/* MX (microscaling, per 32 consecutive values of a view): exponent e =    */
/* floor(log2(block max |x|)) - emax (emax 8 for e4m3, 2 for e2m1),        */
/* clamped to [-127, 127] (-127 for an all-zero block), scale byte e + 127 */
/* into `scale` (uint8 [n][dim/32]); codes round(x / 2^e) to the element   */
/* format (nearest, ties to even, saturating).  dst is [n][dim] bytes      */
/* (MXFP8) or [n][dim/2] bytes (MXFP4).  dim must be a multiple of 32.     */
/* ---------------------------------------------------------------------- */
gift_status gift_quantize_views(const float* src, int64_t n, int32_t dim,
                                int32_t dtype, void* dst, void* scale,
                                void* stream);

/* ---------------------------------------------------------------------- */
/* Exhaustive multi-view matching, Eq. 3 (Sec. 2.3):                      */
/*   S(x_q, x_p) = (1/m) sum_{i<m} max_{j<Nv} s(q_i, p_j),                 */
/* s = cosine similarity = dot product of the unit-norm views, m = number  */
/* of the query's views.  Every database shape is scored in `db->dtype`    */
/* (scales applied per pair before the max), the top `rescore_r` shapes    */
/* by (score desc, id asc) are rescored exactly from the float32 master,   */
/* and the top `top_k` of those are returned by (exact score desc, id asc).*/
/*   ids    [n_queries][top_k] int32, scores [n_queries][top_k] float32    */
/*   flags  [n_queries] int32 or NULL: bit 0 set when the returned list is  */
/*          provably the exact top_k over all N shapes (no shape outside   */
/*          the rescored set can belong to it, given the error bound of    */
/*          the first-pass dtype for this query's own view count, so a     */
/*          query's flag does not depend on the rest of its batch).  A set */
/*          bit is sound; a clear bit claims nothing.                      */
/* Requires top_k <= rescore_r <= min(1024, N).                             */
/* ---------------------------------------------------------------------- */
size_t gift_query_exhaustive_workspace(const gift_views* db,
                                       const gift_queries* q,
                                       int32_t top_k, int32_t rescore_r);
gift_status gift_query_exhaustive(const gift_views* db, const gift_queries* q,
                                  int32_t top_k, int32_t rescore_r,
                                  int32_t* ids, float* scores, int32_t* flags,
                                  void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* gift_query_exhaustive without a workspace argument and without device   */
/* allocation, for callers that cannot allocate (code under HIP graph       */
/* capture, tight serving loops, harnesses that forbid hipMalloc).  Same    */
/* arguments, results, flags and errors as gift_query_exhaustive; its      */
/* scratch is one static device array of GIFT_STATIC_SCRATCH_BYTES (64     */
/* MiB) per device, which every device that runs this call holds until the */
/* process ends.  The first call on a device looks up that array's address */
/* (hipGetSymbolAddress) with the device current; no call allocates.        */
/* gift_query_exhaustive_static_bytes returns the scratch a batch needs     */
/* (= gift_query_exhaustive_workspace); a batch needing more than          */
/* GIFT_STATIC_SCRATCH_BYTES returns GIFT_ECAPACITY before any device work */
/* (e.g. one 64-view query fits up to about 250,000 shapes).  All calls on */
/* one device share its array: calls that overlap on one device (two       */
/* streams, or two threads) RACE and must be serialised by the caller.     */
/* ---------------------------------------------------------------------- */
#define GIFT_STATIC_SCRATCH_BYTES (64u << 20)
size_t gift_query_exhaustive_static_bytes(const gift_views* db, const gift_queries* q,
                                          int32_t top_k, int32_t rescore_r);
gift_status gift_query_exhaustive_static(const gift_views* db, const gift_queries* q,
                                         int32_t top_k, int32_t rescore_r, int32_t* ids,
                                         float* scores, int32_t* flags, void* stream);

/* Full score matrix of the first pass of gift_query_exhaustive (Eq. 3 in   */
/* db->dtype), for inspection: scores [n_queries][n_shapes] float32.        */
size_t gift_score_exhaustive_workspace(const gift_views* db,
                                       const gift_queries* q);
gift_status gift_score_exhaustive(const gift_views* db, const gift_queries* q,
                                  float* scores, void* ws, size_t ws_bytes,
                                  void* stream);

/* ---------------------------------------------------------------------- */
/* Quantizer c(x) with Multiple Assignment (Sec. 2.3):                     */
/*   c(x) = argmin_k ||x - b_k||^2 over the vocabulary B = {b_1..b_K};     */
/* words[r][a] is the a-th nearest codeword of row r of x [n][dim] by      */
/* (exact distance, index), a < ma.  Decided on the exact distance over    */
/* the float32 inputs (float32 MFMA distances, compensated re-evaluation   */
/* of every codeword within the float32 error bound of the ma-th best).    */
/* codebook [K][dim] float32, K <= 16384, ma <= min(8, K).                 */
/* n_uncertified: device int32 or NULL; receives the number of rows with   */
/* more than 256 codewords inside that bound (their words may then not be  */
/* exact; 0 in practice).                                                 */
/* ---------------------------------------------------------------------- */
size_t gift_assign_workspace(int64_t n, int32_t dim, int32_t K, int32_t ma);
gift_status gift_assign(const float* x, int64_t n, int32_t dim,
                        const float* codebook, int32_t K, int32_t ma,
                        int32_t* words, int32_t* n_uncertified,
                        void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Vocabulary by k-means (Sec. 2.3; building it is the main offline cost   */
/* after CNN training, Sec. 3.4).  Lloyd iterations from the K training    */
/* rows init_idx (host int64[K]): assign every row with gift_assign        */
/* (ma = 1); each centroid becomes the float64 sum of its members in       */
/* ascending row order divided in float64 and rounded once to float32; an  */
/* empty cluster keeps its centroid; stop when no assignment changes or    */
/* after max_iter updates.  codebook [K][dim] and assign [n] receive the   */
/* final state; *iters_run (host) the number of updates.  SYNCHRONISES     */
/* `stream` once per iteration.  Returns GIFT_ECAPACITY if an assignment   */
/* could not be certified.                                                */
/* ---------------------------------------------------------------------- */
size_t gift_build_codebook_workspace(int64_t n, int32_t dim, int32_t K);
gift_status gift_build_codebook(const float* train, int64_t n, int32_t dim,
                                int32_t K, const int64_t* init_idx,
                                int32_t max_iter, float* codebook,
                                int32_t* assign, int32_t* iters_run,
                                void* ws, size_t ws_bytes, void* stream);

/* The first inverted file (Sec. 2.3, Fig. 2): K lists; list w holds, in   */
/* ascending (shape, view) order, every database view with w among its ma  */
/* nearest codewords, as (shape id, view index).                          */
typedef struct gift_fif {
  const float*   codebook;    /* [K][dim] float32                             */
  int32_t        K;
  int32_t        ma;          /* codewords per database view                  */
  int64_t        n_entries;   /* = ma * n_shapes * n_views                    */
  const int64_t* offsets;     /* [K+1]: list w is entries [offsets[w], offsets[w+1]) */
  const int32_t* entry_shape; /* [n_entries] shape id p                        */
  const int32_t* entry_view;  /* [n_entries] view index j in 0..n_views-1      */
  const int32_t* view_words;  /* [n_shapes * n_views][ma] words of each view   */
} gift_fif;

/* Builds the F-IF of `db` (which needs `master`) for a codebook: fills     */
/* offsets [K+1], entry_shape / entry_view [ma*N*Nv] and view_words          */
/* [N*Nv][ma].  SYNCHRONISES `stream`; GIFT_ECAPACITY as gift_build_codebook. */
size_t gift_build_fif_workspace(const gift_views* db, int32_t K, int32_t ma);
gift_status gift_build_fif(const gift_views* db, const float* codebook,
                           int32_t K, int32_t ma, int64_t* offsets,
                           int32_t* entry_shape, int32_t* entry_view,
                           int32_t* view_words, void* ws, size_t ws_bytes,
                           void* stream);

/* ---------------------------------------------------------------------- */
/* Inverted-file matching, Eq. 4 (Sec. 2.3):                              */
/*   S_F(x_q, x_p) = (1/m) sum_i max_j s(q_i, p_j) * delta(c(q_i), p_j),   */
/* where a query view is hard-assigned to its nearest word c(q_i) and      */
/* delta is 1 when that word is among the ma words of p_j; a query view    */
/* with no matching view of p contributes 0.  Only the lists of the        */
/* batch's words are scanned.  Ranking, rescore and flags as               */
/* gift_query_exhaustive (the rescore evaluates Eq. 4 exactly); flags bit  */
/* 1 marks a batch in which a query word could not be certified.           */
/* ---------------------------------------------------------------------- */
size_t gift_query_fif_workspace(const gift_views* db, const gift_fif* fif,
                                const gift_queries* q, int32_t top_k,
                                int32_t rescore_r);
gift_status gift_query_fif(const gift_views* db, const gift_fif* fif,
                           const gift_queries* q, int32_t top_k,
                           int32_t rescore_r, int32_t* ids, float* scores,
                           int32_t* flags, void* ws, size_t ws_bytes,
                           void* stream);

/* First-pass Eq. 4 scores [n_queries][n_shapes] float32 in db->dtype and,  */
/* if qwords != NULL, the word of every query view [total_views] int32.     */
size_t gift_score_fif_workspace(const gift_views* db, const gift_fif* fif,
                                const gift_queries* q);
gift_status gift_score_fif(const gift_views* db, const gift_fif* fif,
                           const gift_queries* q, float* scores,
                           int32_t* qwords, void* ws, size_t ws_bytes,
                           void* stream);

/* ---------------------------------------------------------------------- */
/* The second inverted file (Sec. 2.4, Eq. 7, Fig. 3).  Input: for every   */
/* database shape p its neighbour list nbr_ids / nbr_scores [N][k1] (the   */
/* shape's top-k1 by Eq. 3 or Eq. 4, itself included; ids < 0 are padding) */
/* which defines the sparse activation F_p[i] = S(x_p, x_i) for i in the   */
/* list.  Output: l1 [N][2] = ||F_p||_1 as an unevaluated float pair       */
/* hi + lo (the sigma-count that Eq. 14 pre-computes offline), and the     */
/* postings in CSR by coordinate: post_off [N+1]; entry i lists, in        */
/* ascending p, every shape p with a non-zero membership F_p[i] as         */
/* (post_id = p, post_val = F_p[i]); post_id / post_val need room for N*k1 */
/* entries, post_off[N] is the count used.                                */
/* ---------------------------------------------------------------------- */
size_t gift_build_sif_workspace(int64_t n_shapes);
gift_status gift_build_sif(int64_t n_shapes, int32_t k1, const int32_t* nbr_ids,
                           const float* nbr_scores, float* l1, int64_t* post_off,
                           int32_t* post_id, float* post_val, void* ws,
                           size_t ws_bytes, void* stream);

/* Neighbour augmentation (Sec. 2.4.1, Eq. 10): sparse activation rows     */
/* replaced by the mean of the rows of their top-k2 neighbours,            */
/*   F_b := (1 / n_b) * sum over members i of F_i.                         */
/* The table nbr_ids / nbr_scores [N][k1] holds F_i of every database shape */
/* as a list (ids < 0 are padding).  Member j of output row b is table row */
/* members[b][j] (ids < 0 skipped; a database shape lists itself first, so */
/* k2 = 1 leaves it unchanged); when own_ids / own_scores [n_rows][k_own]  */
/* are given, that list is one more member (a query outside the database). */
/* n_b = number of members.  The right-hand side uses the un-augmented     */
/* rows.  Output rows out_ids / out_scores [n_rows][k_out] list the        */
/* coordinates in ascending id with their averaged memberships, padded     */
/* with (-1, 0) (rows longer than k_out are cut); n_members [n_rows] (or    */
/* NULL) receives n_b, so a query's self membership becomes q_self / n_b.  */
/* Requires k2 * k1 + k_own <= 1024.                                       */
gift_status gift_augment_neighbours(int64_t n_shapes, int32_t k1,
                                   const int32_t* nbr_ids,
                                   const float* nbr_scores, int32_t n_rows,
                                   const int32_t* members, int32_t k2,
                                   const int32_t* own_ids,
                                   const float* own_scores, int32_t k_own,
                                   int32_t* out_ids, float* out_scores,
                                   int32_t k_out, int32_t* n_members,
                                   void* stream);

/* Aggregated contextual activation (Sec. 2.4, Eq. 9): the element-wise    */
/* generalised mean with exponent alpha of two sparse activations of the   */
/* same shapes from two similarity measures,                               */
/*   F = ((F1^alpha + F2^alpha) / 2)^(1/alpha),                            */
/* over the union of each row's coordinates (a coordinate missing from one */
/* row contributes 0).  Rows ids1/scores1 [n_rows][k_a] and ids2/scores2    */
/* [n_rows][k_b] (ids < 0 skipped, ids distinct within a row); output       */
/* [n_rows][k_out] in ascending id, padded with (-1, 0).  Neighbour        */
/* co-augmentation (Eq. 11) is gift_augment_neighbours with the other      */
/* measure's neighbour ids as members.  alpha > 0; k_a + k_b <= 1024.      */
gift_status gift_fuse_activations(int32_t n_rows, const int32_t* ids1,
                                  const float* scores1, int32_t k_a,
                                  const int32_t* ids2, const float* scores2,
                                  int32_t k_b, float alpha, int32_t* out_ids,
                                  float* out_scores, int32_t k_out,
                                  void* stream);

/* Self membership of queries outside the database through Eq. 11 and      */
/* Eq. 9.  Such a query joins its own neighbour set under each measure     */
/* with membership self1[b] / self2[b] (1 for unit-norm views, the Eq. 3   */
/* self score); gift_augment_neighbours averages its row over n1[b] / n2[b] */
/* members (its n_members output), so the own membership becomes self / n; */
/* out[b] is the generalised mean with exponent alpha of the two, as       */
/* gift_fuse_activations forms it for every other coordinate.  It is the   */
/* q_self of gift_rerank_sif for the fused activation.  All arrays device, */
/* [n_rows]; n <= 0 counts as membership 0.  alpha > 0.                    */
gift_status gift_fuse_self(int32_t n_rows, const float* self1, const int32_t* n1,
                           const float* self2, const int32_t* n2, float alpha, float* out,
                           void* stream);

/* Re-ranking by Eq. 8 evaluated through the S-IF (Eq. 13 and 14):        */
/*   S'(q, p) = sum_i min(F_q[i], F_p[i]) / (||F_q||_1 + ||F_p||_1 - num),  */
/* the numerator taken over the coordinates where both are non-zero.  The  */
/* query's activation is q_ids / q_scores [n_queries][k1] (ids < 0 skipped)*/
/* plus a membership q_self[b] of the query in its own neighbour set (a    */
/* query outside the database has no coordinate of its own, so q_self only */
/* enters ||F_q||_1; pass 0, or q_self = NULL, for a database shape whose   */
/* own id is in q_ids).  Returns the top_k shapes by (S' desc, id asc);    */
/* shapes sharing no coordinate score 0 and fill the list in id order.     */
/* S' is formed in compensated arithmetic.  The result is exact for any    */
/* number of postings: a query whose coordinates hold more than 4096       */
/* postings is processed in several ranges of shape ids, each of at most   */
/* 4096 postings.  flags [n_queries] (or NULL): bit 0 always set (exact),  */
/* bit 1 set when the query took more than one range.                     */
/* Requires 1 <= top_k <= min(n_shapes, 1024), 1 <= k1 <= 256.             */
/* ---------------------------------------------------------------------- */
gift_status gift_rerank_sif(int64_t n_shapes, const float* l1,
                            const int64_t* post_off, const int32_t* post_id,
                            const float* post_val, int32_t n_queries,
                            int32_t k1, const int32_t* q_ids,
                            const float* q_scores, const float* q_self,
                            int32_t top_k, int32_t* ids, float* scores,
                            int32_t* flags, void* stream);

/* ---------------------------------------------------------------------- */
/* Batch plans for the F-IF path (Eq. 4, then the exact rescore and        */
/* ranking of gift_query_fif).  A plan fixes the database, the index and   */
/* capacities (max_queries, max_views in total, max_views_per_query, the   */
/* last checked at creation only: certificates use each query's own view   */
/* count) and                                                              */
/* binds caller-owned device buffers: q_views [max_views][dim] float32 and */
/* q_offsets [max_queries + 1] (the batch input, written by the caller     */
/* before each run; q_offsets[0] = 0), and the outputs ids / scores        */
/* [max_queries][top_k] and flags [max_queries] (NULL allowed).  The first */
/* pass runs as ONE persistent kernel whose blocks take work items         */
/* (split and quantize, dot tiles that also clear the match buffer, word  */
/* selection, grouping, list tiles, per-query means) in order from a      */
/* device queue; it is followed by                                        */
/* the selection, rescore and final-ranking kernels, and the whole         */
/* sequence is captured once into a HIP graph.                              */
/* gift_fif_plan_run(n_queries, n_views)                                   */
/* launches that graph for a batch occupying the first n_queries slots and  */
/* n_views rows; outputs of unused slots are unspecified.  The first-pass */
/* scores, ids, scores and flags equal those of gift_query_fif on the same */
/* batch (the same tiles in the same order) under the default tuning.     */
/* `tuning` (NULL: the defaults) sets the persistent grid (blocks_per_cu,   */
/* 1 or 2; default 2), the list entries per scan item (list_tile, 32..128  */
/* in steps of 32; default 128) and the largest query-view group that takes */
/* the narrow scan tile (narrow_max, 0, 16 or 32; default 32) and where   */
/* the codeword GEMM runs (gemm, see gift_plan_tuning).  Every             */
/* tuning gives the same ids and exact scores; a first-pass value, and so  */
/* a flag, may differ in the last bits between tunings.  The workspace     */
/* size depends on list_tile.  Create SYNCHRONISES `stream` (which must be a */
/* non-default stream not being captured); run is asynchronous.  A plan is */
/* not thread-safe and its runs on different streams must not overlap.     */
/* gift_fif_plan_first_pass copies the first-pass Eq. 4 scores of the     */
/* last run's first n_queries slots to out [n_queries][n_shapes] float32   */
/* (device; asynchronous on `stream`), for inspection.                     */
/* gift_fif_plan_error (SYNCHRONISES) returns 1 if a queue wait of the     */
/* last run hit its time limit (results invalid), else 0.                  */
/* gift_fif_plan_phase_us (SYNCHRONISES) writes, for the last run, the     */
/* block-microseconds spent in each phase of the persistent kernel (sum    */
/* over blocks of the wall time from the end of an item's wait for its     */
/* inputs to the end of the item): out[9] = split and quantize, codeword   */
/* dots, clear (no items of its own: the dot-tile items clear the match  */
/* buffer, so it reads 0), word selection, word offsets, grouping,        */
/* active-tile listing, list scan, per-query mean.                         */
/* gift_fif_plan_phase_end_us (SYNCHRONISES) writes, for the last run and  */
/* the same nine phases, the microseconds from the start of the run's      */
/* queue reset to the end of the phase's last item (0: no item).           */
/* ---------------------------------------------------------------------- */
typedef struct gift_fif_plan gift_fif_plan;
typedef struct gift_plan_tuning {
  int32_t blocks_per_cu;  /* persistent blocks per CU: 1 or 2                */
  int32_t list_tile;      /* list entries per scan item: 32, 64, 96 or 128   */
  int32_t narrow_max;     /* groups of at most this many query views take
                             the narrow scan tile: 0 (none), 16 or 32        */
  int32_t gemm;           /* codeword GEMM: 0 auto (2 when max_views >=
                             16384, else 1), 1 dot tiles inside the
                             persistent kernel, 2 a separate 256 x 256 GEMM
                             kernel before it (which also clears the match
                             buffer)                                         */
} gift_plan_tuning;
size_t gift_fif_plan_workspace(const gift_views* db, const gift_fif* fif,
                               int32_t max_queries, int64_t max_views,
                               int32_t top_k, int32_t rescore_r,
                               const gift_plan_tuning* tuning);
gift_status gift_fif_plan_create(const gift_views* db, const gift_fif* fif,
                                 int32_t max_queries, int64_t max_views,
                                 int32_t max_views_per_query, int32_t top_k,
                                 int32_t rescore_r, const float* q_views,
                                 int32_t* q_offsets, int32_t* ids,
                                 float* scores, int32_t* flags,
                                 const gift_plan_tuning* tuning, void* ws,
                                 size_t ws_bytes, void* stream,
                                 gift_fif_plan** plan);
gift_status gift_fif_plan_run(gift_fif_plan* plan, int32_t n_queries,
                              int64_t n_views, void* stream);
/* One serving launch in one call, for host loops that stage each batch   */
/* in pinned host memory: copies n_views x dim query views and the        */
/* n_queries + 1 offsets from the host buffers into the plan's q_views /  */
/* q_offsets, runs the plan (as gift_fif_plan_run), then, when l1 is not  */
/* NULL, re-ranks the plan's ids / scores [n_queries][top_k of the plan]  */
/* by Eq. 8 as gift_rerank_sif does (the S-IF arrays, q_self and top_k as */
/* there; rr_ids / rr_scores [n_queries][top_k] and rr_flags [n_queries]  */
/* are device buffers the caller owns), and copies the final ids, scores  */
/* and flags to host_ids / host_scores / host_flags ([n_queries][k] with  */
/* k the re-rank's top_k, else the plan's; host_flags may be NULL without */
/* a re-rank).  Everything is queued on `stream`; the caller keeps the    */
/* host buffers alive and unmodified until the stream has passed the     */
/* copies (record an event after the call).  GIFT_EINVAL for a null plan  */
/* or host buffer or incomplete re-rank arguments, GIFT_ECAPACITY as for   */
/* gift_fif_plan_run; n_queries == 0 queues nothing.                      */
gift_status gift_fif_plan_serve(gift_fif_plan* plan, const float* host_views,
                                const int32_t* host_offsets, int32_t n_queries,
                                int64_t n_views, int64_t n_shapes, const float* l1,
                                const int64_t* post_off, const int32_t* post_id,
                                const float* post_val, const float* q_self,
                                int32_t top_k, int32_t* rr_ids, float* rr_scores,
                                int32_t* rr_flags, int32_t* host_ids, float* host_scores,
                                int32_t* host_flags, void* stream);
/* The same sequence launched kernel by kernel (no graph), for comparison. */
gift_status gift_fif_plan_run_eager(gift_fif_plan* plan, int32_t n_queries,
                                    int64_t n_views, void* stream);
gift_status gift_fif_plan_first_pass(gift_fif_plan* plan, int32_t n_queries, float* out,
                                     void* stream);
gift_status gift_fif_plan_error(gift_fif_plan* plan, int32_t* err,
                                void* stream);
gift_status gift_fif_plan_phase_us(gift_fif_plan* plan, double* out /* host [9] */,
                                   void* stream);
gift_status gift_fif_plan_phase_end_us(gift_fif_plan* plan, double* out /* host [9] */,
                                       void* stream);
gift_status gift_fif_plan_destroy(gift_fif_plan* plan);

/* ---------------------------------------------------------------------- */
/* Asynchronous copy of `bytes` bytes from src to dst on `stream`, each    */
/* side host or device (the direction follows from the pointers; host     */
/* memory must be pinned for the copy to stay asynchronous).  For callers */
/* that stage batches through pinned host buffers, such as a serving loop,*/
/* one call per buffer without a framework copy around it.  The caller    */
/* owns both buffers and keeps them alive until the stream has passed the */
/* copy.  GIFT_EINVAL for a null pointer with bytes > 0; GIFT_EHIP when   */
/* the copy cannot be queued.  bytes == 0 does nothing.                    */
/* ---------------------------------------------------------------------- */
gift_status gift_copy_async(void* dst, const void* src, size_t bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Tuning of the first-pass scorer (host, process-wide, not thread-safe).  */
/* tile (BF16 / FP8 storage; float32 always uses 128 x 128 and MX storage */
/* 256 x 128), 0..8: for 0..3, bit 0 selects 256 database rows x 256 query */
/* views per block instead of 256 x 128 and bit 1 the pipelined main loop */
/* with direct global-to-LDS loads in 64-byte sub-tiles (4 waves); 4 is   */
/* the 256 x 256 direct-load tile with 8 waves (two per SIMD); 5 and 6 are */
/* 3 and 4 with 128-byte sub-tiles; 7 is 6 with three LDS stages of query */
/* rows; 8 is 6 as a persistent kernel (one block per CU walking the      */
/* tiles, the next tile's first sub-tile loading during the epilogue).    */
/* A stored row that is no whole number of sub-tiles falls back to a tile */
/* it holds (6, 7, 8 -> 4 -> 1; 5 -> 3 -> 1).                             */
/* The default is 8 with group 32.  group: number of database             */
/* row tiles that share one sweep over the query tiles in the launch order */
/* (blocks go to the 8 XCDs round-robin, so multiples of 8 keep each       */
/* database tile on one XCD).  gift_autotune_score times every (tile,      */
/* group) pair of the given lists on this workload (reps launches each,   */
/* HIP events on `stream`; SYNCHRONISES), writes the average ms per launch */
/* to ms_out [n_tiles][n_groups] (may be NULL), selects the fastest pair   */
/* and returns it.  Workspace as gift_score_exhaustive.                    */
/* ---------------------------------------------------------------------- */
gift_status gift_set_score_tuning(int32_t dtype, int32_t tile, int32_t group);
gift_status gift_get_score_tuning(int32_t dtype, int32_t* tile, int32_t* group);
gift_status gift_autotune_score(const gift_views* db, const gift_queries* q,
                                const int32_t* tiles, int32_t n_tiles,
                                const int32_t* groups, int32_t n_groups,
                                int32_t reps, float* ms_out,
                                int32_t* best_tile, int32_t* best_group,
                                void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Kernel timing.  gift_profile_enable(capacity > 0) creates `capacity`   */
/* HIP event pairs and from then on brackets each kernel launch of the    */
/* calls above with events recorded on the launch stream (first          */
/* `capacity` launches after a reset); capacity 0 turns timing off and    */
/* frees the events.  gift_profile_read() waits for the recorded events  */
/* of kernel `tag` and returns their summed duration and count.  Tags:   */
/* 0 quantize, 1 score_tiles, 2 reduce_queries, 3 select_top, 4 rescore,  */
/* 5 final_rank, 6 assign, 7 group_queries, 8 fif_scan, 9 rerank_sif.      */
/* Host functions,                                                        */
/* not thread-safe.                                                       */
/* ---------------------------------------------------------------------- */
gift_status gift_profile_enable(int32_t capacity);
gift_status gift_profile_reset(void);
gift_status gift_profile_read(int32_t tag, double* total_ms, int32_t* count);
const char* gift_profile_tag_name(int32_t tag);

/* ---------------------------------------------------------------------- */
/* Measurement probe (not part of the search path): the sustained rate of */
/* one 32 x 32 MFMA kind.  Launches `blocks` blocks of 4 waves; each wave */
/* issues `iters` rounds of 8 independent MFMAs of dtype GIFT_F32         */
/* (32x32x2, 4096 flop each), GIFT_BF16 (32x32x16, 32768 flop) or         */
/* GIFT_FP8E4M3 (32x32x64 e4m3, 131072 flop), on `stream`.  Writes each   */
/* thread's accumulator sum to sink (device, blocks * 256 floats) and, per */
/* block, the clock64() and wall_clock64() deltas of its first wave to    */
/* clocks (device, 2 * blocks), and the wall clock's rate in kHz to       */
/* *wall_khz (host), so delta[0] / delta[1] * wall_khz is the shader      */
/* clock in kHz over that block's loop.  Time the launch with events on   */
/* the same stream.  GIFT_EINVAL for another dtype, a non-positive count  */
/* or a null pointer.                                                     */
/* ---------------------------------------------------------------------- */
gift_status gift_probe_mfma(int32_t dtype, int32_t blocks, int32_t iters, float* sink,
                            uint64_t* clocks, int32_t* wall_khz, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GIFT_H */
