// C ABI entry points: argument validation, workspace layout and the launch
// sequence of each call.  All arithmetic happens in the kernels.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "kernels.h"

namespace gift {

static thread_local char g_err[512] = "";

gift_status fail(gift_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

// ---------------------------------------------------------------- profiling
// Optional HIP-event brackets around each kernel launch, on the launch
// stream, so a caller can read per-kernel device time.  Off by default.
enum ProfTag { P_QUANT = 0, P_SCORE, P_REDUCE, P_SELECT, P_RESCORE, P_FINAL, P_NTAGS };
static const char* kTagNames[P_NTAGS] = {"quantize", "score_tiles", "reduce_queries",
                                         "select_top", "rescore", "final_rank"};
struct ProfSlot { hipEvent_t a, b; int tag; };
static ProfSlot* g_prof = nullptr;
static int g_prof_cap = 0, g_prof_used = 0, g_prof_on = 0;

static void prof_begin(int tag, hipStream_t st) {
  if (!g_prof_on || g_prof_used >= g_prof_cap) return;
  g_prof[g_prof_used].tag = tag;
  (void)hipEventRecord(g_prof[g_prof_used].a, st);
}
static void prof_end(hipStream_t st) {
  if (!g_prof_on || g_prof_used >= g_prof_cap) return;
  (void)hipEventRecord(g_prof[g_prof_used].b, st);
  ++g_prof_used;
}

static const double U32 = 5.9604644775390625e-08;  // 2^-24

// gamma_n = n u / (1 - n u), the classic bound on an n-term float32 sum.
static double gamma_n(double n) { return n * U32 / (1.0 - n * U32); }

// Bound on |float32 dot - exact dot| of two unit-norm views in the rescore
// kernel: a fresh partial sum per 32 values, added into a running total.
static float rescore_dot_err(int dim) {
  return (float)(gamma_n(32.0 + dim / 32 + 1) * 1.0001);
}

// Bound on |first-pass score - exact Eq. 3 score| for unit-norm views.
// Storage rounding: each stored value is within u_s of the scaled value
// (u_s = 2^-8 for BF16, 2^-4 for e4m3), so a product is within
// 2 u_s + u_s^2 relative; the MFMA accumulation is charged 2*dim roundings;
// the mean over at most max_m views adds gamma_(max_m + 1).
static float first_pass_err(int dtype, int dim, int max_m) {
  double us = dtype == GIFT_BF16 ? 1.0 / 256 : dtype == GIFT_FP8E4M3 ? 1.0 / 16 : 0.0;
  double e = (2 * us + us * us) + gamma_n(2.0 * dim + 4) + gamma_n(max_m + 2.0);
  return (float)(e * 1.001);
}

static gift_status check_views(const gift_views* db) {
  GIFT_CHECK(db != nullptr && db->data != nullptr, GIFT_EINVAL, "null database views");
  GIFT_CHECK(db->dtype == GIFT_F32 || db->dtype == GIFT_BF16 || db->dtype == GIFT_FP8E4M3,
             GIFT_EUNSUPPORTED, "unsupported dtype %d", db->dtype);
  GIFT_CHECK(db->n_views >= 1 && db->n_views <= 64, GIFT_EUNSUPPORTED,
             "n_views must be in 1..64 (got %d)", db->n_views);
  GIFT_CHECK(db->n_shapes >= 1 && db->n_shapes < ((int64_t)1 << 31), GIFT_EINVAL,
             "n_shapes out of range");
  GIFT_CHECK(db->dim >= 32 && db->dim % 32 == 0, GIFT_EUNSUPPORTED,
             "dim must be a positive multiple of 32 (got %d)", db->dim);
  GIFT_CHECK(db->dtype == GIFT_F32 || db->scale != nullptr, GIFT_EINVAL,
             "BF16/FP8 views need per-view scales");
  return GIFT_OK;
}

static gift_status check_queries(const gift_queries* q, int dim) {
  (void)dim;
  GIFT_CHECK(q != nullptr && q->views != nullptr && q->offsets != nullptr, GIFT_EINVAL,
             "null queries");
  GIFT_CHECK(q->n_queries >= 1, GIFT_EINVAL, "n_queries must be >= 1");
  GIFT_CHECK(q->total_views >= 1 && q->total_views < ((int64_t)1 << 31), GIFT_EINVAL,
             "total_views out of range");
  GIFT_CHECK(q->max_views >= 1 && q->max_views <= q->total_views, GIFT_EINVAL,
             "max_views out of range");
  return GIFT_OK;
}

struct ExhaustiveWs {
  void* qcodes;
  float* qscale;
  float* mbuf;
  float* S;
  int32_t* cand;
  float* cand_s;
  float* s_hi;
  float* s_lo;
  size_t bytes;
};

static ExhaustiveWs carve_exhaustive(void* base, const gift_views* db,
                                     const gift_queries* q, int r) {
  Carver c(base);
  ExhaustiveWs w{};
  const int64_t tq = q->total_views;
  if (db->dtype != GIFT_F32) {
    w.qcodes = c.take<uint8_t>((size_t)tq * db->dim * elem_bytes(db->dtype));
    w.qscale = c.take<float>((size_t)tq);
  }
  w.mbuf = c.take<float>((size_t)db->n_shapes * tq);
  w.S = c.take<float>((size_t)q->n_queries * db->n_shapes);
  if (r > 0) {
    w.cand = c.take<int32_t>((size_t)q->n_queries * r);
    w.cand_s = c.take<float>((size_t)q->n_queries * r);
    w.s_hi = c.take<float>((size_t)q->n_queries * r);
    w.s_lo = c.take<float>((size_t)q->n_queries * r);
  }
  w.bytes = c.bytes();
  return w;
}

// Eq. 3 in the storage dtype for every (query, shape) into w.S.
static gift_status first_pass(const gift_views* db, const gift_queries* q,
                              const ExhaustiveWs& w, hipStream_t st) {
  const void* qv = q->views;
  const float* qs = nullptr;
  if (db->dtype != GIFT_F32) {
    prof_begin(P_QUANT, st);
    launch_quantize(q->views, q->total_views, db->dim, db->dtype, w.qcodes, w.qscale, st);
    prof_end(st);
    GIFT_LAUNCHED();
    qv = w.qcodes;
    qs = w.qscale;
  }
  prof_begin(P_SCORE, st);
  gift_status s = launch_score_tiles(db, qv, qs, q->total_views, w.mbuf, q->total_views, st);
  prof_end(st);
  if (s != GIFT_OK) return s;
  prof_begin(P_REDUCE, st);
  launch_reduce_queries(w.mbuf, q->total_views, db->n_shapes, q->offsets, q->n_queries, w.S, st);
  prof_end(st);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

}  // namespace gift

using namespace gift;

extern "C" {

const char* gift_version(void) { return "gift-mi355x 0.1 (gfx950)"; }

const char* gift_last_error(void) { return g_err; }

gift_status gift_profile_enable(int32_t capacity) {
  for (int i = 0; i < g_prof_cap; ++i) {
    (void)hipEventDestroy(g_prof[i].a);
    (void)hipEventDestroy(g_prof[i].b);
  }
  delete[] g_prof;
  g_prof = nullptr;
  g_prof_cap = g_prof_used = g_prof_on = 0;
  if (capacity <= 0) return GIFT_OK;
  g_prof = new ProfSlot[capacity];
  for (int i = 0; i < capacity; ++i) {
    GIFT_HIP(hipEventCreate(&g_prof[i].a));
    GIFT_HIP(hipEventCreate(&g_prof[i].b));
    g_prof_cap = i + 1;
  }
  g_prof_on = 1;
  return GIFT_OK;
}

const char* gift_profile_tag_name(int32_t tag) {
  return (tag >= 0 && tag < P_NTAGS) ? kTagNames[tag] : "";
}

gift_status gift_profile_read(int32_t tag, double* total_ms, int32_t* count) {
  GIFT_CHECK(total_ms && count, GIFT_EINVAL, "null outputs");
  double tot = 0;
  int n = 0;
  for (int i = 0; i < g_prof_used; ++i) {
    if (g_prof[i].tag != tag) continue;
    GIFT_HIP(hipEventSynchronize(g_prof[i].b));
    float ms = 0.f;
    GIFT_HIP(hipEventElapsedTime(&ms, g_prof[i].a, g_prof[i].b));
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *count = n;
  return GIFT_OK;
}

gift_status gift_profile_reset(void) {
  g_prof_used = 0;
  return GIFT_OK;
}

gift_status gift_quantize_views(const float* src, int64_t n, int32_t dim,
                                int32_t dtype, void* dst, float* scale,
                                void* stream) {
  GIFT_CHECK(src && dst && scale, GIFT_EINVAL, "null pointer");
  GIFT_CHECK(n >= 0 && dim >= 1, GIFT_EINVAL, "bad size");
  GIFT_CHECK(dtype == GIFT_BF16 || dtype == GIFT_FP8E4M3, GIFT_EUNSUPPORTED,
             "quantize target must be BF16 or FP8E4M3");
  launch_quantize(src, n, dim, dtype, dst, scale, (hipStream_t)stream);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

size_t gift_score_exhaustive_workspace(const gift_views* db, const gift_queries* q) {
  if (check_views(db) != GIFT_OK || check_queries(q, db->dim) != GIFT_OK) return 0;
  return carve_exhaustive(nullptr, db, q, 0).bytes;
}

gift_status gift_score_exhaustive(const gift_views* db, const gift_queries* q,
                                  float* scores, void* ws, size_t ws_bytes,
                                  void* stream) {
  gift_status s = check_views(db);
  if (s != GIFT_OK) return s;
  if ((s = check_queries(q, db->dim)) != GIFT_OK) return s;
  GIFT_CHECK(scores != nullptr, GIFT_EINVAL, "null scores");
  ExhaustiveWs w = carve_exhaustive(ws, db, q, 0);
  GIFT_CHECK(ws != nullptr && ws_bytes >= w.bytes, GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", w.bytes, ws_bytes);
  w.S = scores;  // write the matrix straight into the caller's buffer
  return first_pass(db, q, w, (hipStream_t)stream);
}

size_t gift_query_exhaustive_workspace(const gift_views* db, const gift_queries* q,
                                       int32_t top_k, int32_t rescore_r) {
  (void)top_k;
  if (check_views(db) != GIFT_OK || check_queries(q, db->dim) != GIFT_OK) return 0;
  return carve_exhaustive(nullptr, db, q, rescore_r > 0 ? rescore_r : 1).bytes;
}

gift_status gift_query_exhaustive(const gift_views* db, const gift_queries* q,
                                  int32_t top_k, int32_t rescore_r,
                                  int32_t* ids, float* scores, int32_t* flags,
                                  void* ws, size_t ws_bytes, void* stream) {
  gift_status s = check_views(db);
  if (s != GIFT_OK) return s;
  if ((s = check_queries(q, db->dim)) != GIFT_OK) return s;
  GIFT_CHECK(ids && scores, GIFT_EINVAL, "null outputs");
  GIFT_CHECK(top_k >= 1 && top_k <= rescore_r && rescore_r <= 1024 &&
                 (int64_t)rescore_r <= db->n_shapes,
             GIFT_EINVAL, "need 1 <= top_k <= rescore_r <= min(1024, N)");
  GIFT_CHECK(db->master != nullptr, GIFT_EINVAL, "the exact rescore needs float32 master views");
  const hipStream_t st = (hipStream_t)stream;
  ExhaustiveWs w = carve_exhaustive(ws, db, q, rescore_r);
  GIFT_CHECK(ws != nullptr && ws_bytes >= w.bytes, GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", w.bytes, ws_bytes);
  if ((s = first_pass(db, q, w, st)) != GIFT_OK) return s;
  prof_begin(P_SELECT, st);
  launch_select_top(w.S, db->n_shapes, q->n_queries, rescore_r, w.cand, w.cand_s, st);
  prof_end(st);
  GIFT_LAUNCHED();
  prof_begin(P_RESCORE, st);
  launch_rescore(db->master, db->n_views, db->dim, q->views, q->offsets, q->n_queries,
                 q->max_views, w.cand, rescore_r, rescore_dot_err(db->dim), w.s_hi, w.s_lo, st);
  prof_end(st);
  GIFT_LAUNCHED();
  prof_begin(P_FINAL, st);
  launch_final_rank(w.cand, w.cand_s, w.s_hi, w.s_lo, q->n_queries, rescore_r, top_k,
                    db->n_shapes, first_pass_err(db->dtype, db->dim, q->max_views), ids,
                    scores, flags, st);
  prof_end(st);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

}  // extern "C"
