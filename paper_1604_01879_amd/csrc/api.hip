// C ABI entry points: argument validation, workspace layout and the launch
// sequence of each call.  All arithmetic happens in the kernels.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <set>
#include <utility>

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

gift_status ensure_dynamic_lds(const void* kernel, size_t bytes) {
  static std::mutex mu;
  static std::set<std::pair<const void*, int>> done;
  int dev = 0;
  GIFT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({kernel, dev})) return GIFT_OK;
  GIFT_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done.insert({kernel, dev});
  return GIFT_OK;
}

// ---------------------------------------------------------------- profiling
// Optional HIP-event brackets around each kernel launch, on the launch
// stream, so a caller can read per-kernel device time.  Off by default.
enum ProfTag { P_QUANT = 0, P_SCORE, P_REDUCE, P_SELECT, P_RESCORE, P_FINAL, P_ASSIGN,
               P_GROUP, P_SCAN, P_RERANK, P_NTAGS };
static const char* kTagNames[P_NTAGS] = {"quantize", "score_tiles", "reduce_queries",
                                         "select_top", "rescore", "final_rank", "assign",
                                         "group_queries", "fif_scan", "rerank_sif"};
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

// Bound on |approximate dot - exact dot| of two unit-norm views in the
// rescore kernel.  Splitting x = hi + lo + r (bfloat16 hi, lo; |x - hi| <=
// 2^-8 |x|, |r| <= 2^-16 |x|) and dropping lo.lo', hi.r', r.hi' and smaller
// terms costs at most 3.02 * 2^-16 sum |x y|.  Per 32-value K-tile, 6 BF16
// MFMAs of 16 products each (charged 17 roundings each) go into a fresh
// block that is added into a running total; the summed terms are at most
// 1.02 sum |x y|.  sum |x y| <= 1 for unit-norm views.  The absolute term
// covers values small enough for their low parts to be denormal.
static float rescore_dot_err(int dim) {
  const double split = 3.02 / 65536.0;
  return (float)((split + 1.02 * gamma_n(6.0 * 17 + dim / 32 + 2)) * 1.0001 + 1e-25);
}

// Bound on |first-pass score - exact Eq. 3 / Eq. 4 score| for unit-norm
// views, without the mean's term.  Storage rounding: each stored value is
// within u_s of the scaled value (u_s = 2^-8 for BF16, 2^-4 for e4m3), so a
// product is within 2 u_s + u_s^2 relative; the MFMA accumulation is
// charged 2*dim roundings.  Float32 rows carry no storage error; in the
// Eq. 4 list scan (`list_scan`) their tiles sum each 32-value K-tile into a
// fresh block that is added into the running total, so a product is
// rounded once, passes through at most 32 additions in its block (2 per
// 32x32x2 MFMA, 4 per 16x16x4 MFMA) and at most dim / 32 into the total,
// which 48 + dim / 32 + 2 roundings cover (the absolute term covers
// products flushed to zero).  The final ranking adds the mean over the
// query's own m views, gamma_(m + 2), per query (so a query's certificate
// does not depend on the other queries of its batch), and a 1.001 safety
// factor.
static double first_pass_err(int dtype, int dim, bool list_scan) {
  // MX element errors are relative to the block maximum, not the element
  // (saturation can cost an eighth of it): no useful bound, so never certify
  if (dtype == GIFT_MXFP8 || dtype == GIFT_MXFP4) return 4.0;
  if (dtype == GIFT_F32 && list_scan) return gamma_n(48.0 + (dim + 31) / 32 + 2) * 1.0001 + 1e-25;
  double us = dtype == GIFT_BF16 ? 1.0 / 256 : dtype == GIFT_FP8E4M3 ? 1.0 / 16 : 0.0;
  return (2 * us + us * us) + gamma_n(2.0 * dim + 4);
}

float rescore_dot_error(int dim) { return rescore_dot_err(dim); }
double first_pass_error(int dtype, int dim, bool list_scan) {
  return first_pass_err(dtype, dim, list_scan);
}

// Rows are read with 16-byte vector loads and scales with 4-byte loads.
static bool aligned(const void* p, uintptr_t a) {
  return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0;
}

static gift_status check_views(const gift_views* db) {
  GIFT_CHECK(db != nullptr && db->data != nullptr, GIFT_EINVAL, "null database views");
  GIFT_CHECK(aligned(db->data, 16) && aligned(db->master, 16) && aligned(db->scale, 4),
             GIFT_EINVAL, "views and master views must be 16-byte aligned, scales 4-byte");
  GIFT_CHECK(db->dtype >= GIFT_F32 && db->dtype <= GIFT_MXFP4, GIFT_EUNSUPPORTED,
             "unsupported dtype %d", db->dtype);
  GIFT_CHECK(db->dtype != GIFT_MXFP8 || db->dim % 128 == 0, GIFT_EUNSUPPORTED,
             "MXFP8 storage needs dim a multiple of 128");
  GIFT_CHECK(db->dtype != GIFT_MXFP4 || db->dim % 256 == 0, GIFT_EUNSUPPORTED,
             "MXFP4 storage needs dim a multiple of 256");
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
  GIFT_CHECK(aligned(q->views, 16), GIFT_EINVAL, "query views must be 16-byte aligned");
  GIFT_CHECK(q->n_queries >= 1, GIFT_EINVAL, "n_queries must be >= 1");
  GIFT_CHECK(q->total_views >= 1 && q->total_views < ((int64_t)1 << 31), GIFT_EINVAL,
             "total_views out of range");
  GIFT_CHECK(q->max_views >= 1 && q->max_views <= q->total_views, GIFT_EINVAL,
             "max_views out of range");
  return GIFT_OK;
}

struct ExhaustiveWs {
  void* qcodes;
  void* qscale;
  float* mbuf;
  float* S;
  int32_t* cand;
  float* cand_s;
  void* sel_tmp;  // chunk winners of the top-r selection
  float* s_hi;
  float* s_lo;
  RescoreScratch rs;  // rescore masks, approximate scores, top-k marks
  size_t bytes;
};

static ExhaustiveWs carve_exhaustive(void* base, const gift_views* db,
                                     const gift_queries* q, int r) {
  Carver c(base);
  ExhaustiveWs w{};
  const int64_t tq = q->total_views;
  if (db->dtype != GIFT_F32) {
    w.qcodes = c.take<uint8_t>((size_t)tq * row_bytes_of(db->dtype, db->dim));
    w.qscale = is_mx(db->dtype) ? (void*)c.take<uint8_t>((size_t)tq * (db->dim / 32))
                                : (void*)c.take<float>((size_t)tq);
  }
  w.mbuf = c.take<float>((size_t)db->n_shapes * tq);
  w.S = c.take<float>((size_t)q->n_queries * db->n_shapes);
  if (r > 0) {
    w.cand = c.take<int32_t>((size_t)q->n_queries * r);
    w.cand_s = c.take<float>((size_t)q->n_queries * r);
    w.sel_tmp = c.take<uint8_t>(select_top_ws(db->n_shapes, q->n_queries, r));
    w.s_hi = c.take<float>((size_t)q->n_queries * r);
    w.s_lo = c.take<float>((size_t)q->n_queries * r);
    w.rs = take_rescore(c, q->n_queries, r, q->total_views);
  }
  w.bytes = c.bytes();
  return w;
}

// Eq. 3 in the storage dtype for every (query, shape) into w.S.
static gift_status first_pass(const gift_views* db, const gift_queries* q,
                              const ExhaustiveWs& w, hipStream_t st) {
  const void* qv = q->views;
  const void* qs = nullptr;
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

// ---------------------------------------------------------------- quantizer
struct AssignWs {
  float* D;
  float* nhi;
  float* nlo;
  int32_t* overflow;
  uint8_t* xs;   // BF16-split rows of a chunk
  uint8_t* cbs;  // BF16-split codebook
  int64_t chunk;
};

static int64_t assign_chunk(int64_t n, int K) {
  int64_t c = ((int64_t)1 << 28) / (K > 0 ? K : 1);  // <= 1 GiB of float32 dots
  if (c < 128) c = 128;
  return n < c ? (n > 0 ? n : 1) : c;
}

static AssignWs carve_assign(Carver& c, int64_t n, int K, int dim) {
  AssignWs w{};
  w.chunk = assign_chunk(n, K);
  w.D = c.take<float>((size_t)w.chunk * K);
  w.nhi = c.take<float>((size_t)K);
  w.nlo = c.take<float>((size_t)K);
  w.overflow = c.take<int32_t>(1);
  w.xs = c.take<uint8_t>((size_t)w.chunk * dim * 4);
  w.cbs = c.take<uint8_t>((size_t)K * dim * 4);
  return w;
}

static gift_status check_codebook(const float* cb, int K, int ma, int dim) {
  GIFT_CHECK(cb != nullptr, GIFT_EINVAL, "null codebook");
  GIFT_CHECK(aligned(cb, 16), GIFT_EINVAL, "codebook and training rows must be 16-byte aligned");
  GIFT_CHECK(K >= 1 && K <= 16384, GIFT_EUNSUPPORTED, "K must be in 1..16384 (got %d)", K);
  GIFT_CHECK(ma >= 1 && ma <= 8 && ma <= K, GIFT_EUNSUPPORTED, "ma must be in 1..min(8, K)");
  GIFT_CHECK(dim >= 32 && dim % 32 == 0, GIFT_EUNSUPPORTED, "dim must be a multiple of 32");
  return GIFT_OK;
}

// ---------------------------------------------------------------- F-IF query
struct FifWs {
  int32_t* qwords;
  AssignWs as;
  int64_t* goff;
  int32_t* gitems;
  void* bucket;
  void* qcodes;
  void* qscale;
  uint32_t* mbuf;
  float* S;
  int64_t* tile_off;
  int64_t* tcount;
  int32_t* cand;
  float* cand_s;
  void* sel_tmp;  // chunk winners of the top-r selection
  float* s_hi;
  float* s_lo;
  RescoreScratch rs;  // rescore masks, approximate scores, top-k marks
  size_t bytes;
};

static FifWs carve_fif(void* base, const gift_views* db, const gift_fif* f,
                       const gift_queries* q, int r) {
  Carver c(base);
  FifWs w{};
  const int64_t tq = q->total_views;
  w.qwords = c.take<int32_t>((size_t)tq);
  w.as = carve_assign(c, tq, f->K, db->dim);
  w.goff = c.take<int64_t>((size_t)f->K + 1);
  w.gitems = c.take<int32_t>((size_t)tq);
  w.bucket = c.take<uint8_t>(bucket_sort_ws(tq, f->K));
  if (db->dtype != GIFT_F32) {
    w.qcodes = c.take<uint8_t>((size_t)tq * row_bytes_of(db->dtype, db->dim));
    // per-view float32 scales, or E8M0 rows of dim / 32 bytes (MX)
    w.qscale = c.take<uint8_t>(is_mx(db->dtype) ? (size_t)tq * (db->dim / 32)
                                                : (size_t)tq * sizeof(float));
  }
  w.mbuf = c.take<uint32_t>((size_t)db->n_shapes * tq);
  w.S = c.take<float>((size_t)q->n_queries * db->n_shapes);
  w.tile_off = c.take<int64_t>((size_t)f->K + 1);
  w.tcount = c.take<int64_t>((size_t)f->K);
  if (r > 0) {
    w.cand = c.take<int32_t>((size_t)q->n_queries * r);
    w.cand_s = c.take<float>((size_t)q->n_queries * r);
    w.sel_tmp = c.take<uint8_t>(select_top_ws(db->n_shapes, q->n_queries, r));
    w.s_hi = c.take<float>((size_t)q->n_queries * r);
    w.s_lo = c.take<float>((size_t)q->n_queries * r);
    w.rs = take_rescore(c, q->n_queries, r, q->total_views);
  }
  w.bytes = c.bytes();
  return w;
}

static gift_status check_fif(const gift_fif* f, const gift_views* db) {
  GIFT_CHECK(f != nullptr && f->offsets && f->entry_shape && f->entry_view && f->view_words,
             GIFT_EINVAL, "incomplete F-IF index");
  gift_status s = check_codebook(f->codebook, f->K, f->ma, db->dim);
  if (s != GIFT_OK) return s;
  GIFT_CHECK(f->n_entries == (int64_t)f->ma * db->n_shapes * db->n_views, GIFT_EINVAL,
             "n_entries must be ma * n_shapes * n_views");
  return GIFT_OK;
}

// Eq. 4 first pass for every (query, shape) into w.S (float32).
static gift_status fif_first_pass(const gift_views* db, const gift_fif* f, const gift_queries* q,
                                  const FifWs& w, hipStream_t st) {
  const int64_t tq = q->total_views;
  launch_fill_i32(w.as.overflow, 1, 0, st);
  prof_begin(P_ASSIGN, st);
  gift_status s = launch_assign(q->views, tq, db->dim, f->codebook, f->K, 1, w.qwords, w.as.D,
                                w.as.chunk, w.as.nhi, w.as.nlo, w.as.overflow, w.as.xs, w.as.cbs,
                                st);
  prof_end(st);
  if (s != GIFT_OK) return s;
  prof_begin(P_GROUP, st);
  s = launch_bucket_sort(w.qwords, tq, f->K, w.goff, 0, 1, 1, w.gitems, nullptr, w.bucket, st);
  prof_end(st);
  if (s != GIFT_OK) return s;
  const void* qv = q->views;
  const void* qs = nullptr;
  if (db->dtype != GIFT_F32) {
    prof_begin(P_QUANT, st);
    launch_quantize(q->views, tq, db->dim, db->dtype, w.qcodes, w.qscale, st);
    prof_end(st);
    GIFT_LAUNCHED();
    qv = w.qcodes;
    qs = w.qscale;
  }
  launch_fill_i32(reinterpret_cast<int32_t*>(w.mbuf), db->n_shapes * tq, 0, st);
  GIFT_LAUNCHED();
  prof_begin(P_SCAN, st);
  s = launch_fif_scan(db, f->offsets, f->entry_shape, f->entry_view, f->n_entries, f->K,
                      w.tile_off, w.tcount, w.goff, w.gitems, qv, qs, w.mbuf, db->n_shapes, st);
  prof_end(st);
  if (s != GIFT_OK) return s;
  prof_begin(P_REDUCE, st);
  launch_reduce_fif(w.mbuf, db->n_shapes, db->n_shapes, q->offsets, q->n_queries, w.S, st);
  prof_end(st);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

}  // namespace gift

namespace gift {

// Scratch of gift_query_exhaustive_static.  Each device that runs the call
// holds its own copy until the process ends.  In host code `scratch` only
// names the symbol: its device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and that address is the only one
// host code hands to kernels.
static __device__ __align__(256) uint8_t scratch[GIFT_STATIC_SCRATCH_BYTES];

static gift_status static_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  GIFT_HIP(hipGetDevice(&dev));
  GIFT_CHECK(dev >= 0 && dev < kMaxDevices, GIFT_EUNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(mu);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    GIFT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    GIFT_CHECK(p != nullptr, GIFT_EHIP, "no device address for the static scratch");
    addr[dev] = p;
  }
  *out = addr[dev];
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
                                int32_t dtype, void* dst, void* scale,
                                void* stream) {
  GIFT_CHECK(src && dst && scale, GIFT_EINVAL, "null pointer");
  GIFT_CHECK(n >= 0 && dim >= 1, GIFT_EINVAL, "bad size");
  GIFT_CHECK(dtype == GIFT_BF16 || dtype == GIFT_FP8E4M3 || dtype == GIFT_MXFP8 ||
                 dtype == GIFT_MXFP4,
             GIFT_EUNSUPPORTED, "quantize target must be BF16, FP8E4M3, MXFP8 or MXFP4");
  GIFT_CHECK(!is_mx(dtype) || dim % 32 == 0, GIFT_EUNSUPPORTED, "MX storage needs dim % 32 == 0");
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
  launch_select_top(w.S, db->n_shapes, q->n_queries, rescore_r, nullptr, w.cand, w.cand_s,
                    w.sel_tmp, st);
  prof_end(st);
  GIFT_LAUNCHED();
  prof_begin(P_RESCORE, st);
  launch_rescore(db->master, db->n_views, db->dim, q->views, q->offsets, q->n_queries,
                 q->total_views, w.cand, rescore_r, top_k, rescore_dot_err(db->dim), nullptr,
                 nullptr, 0, nullptr, w.cand_s, first_pass_err(db->dtype, db->dim, false), w.rs, w.s_hi,
                 w.s_lo, st);
  prof_end(st);
  GIFT_LAUNCHED();
  prof_begin(P_FINAL, st);
  launch_final_rank(w.cand, w.cand_s, w.s_hi, w.s_lo, q->n_queries, rescore_r, top_k,
                    db->n_shapes, first_pass_err(db->dtype, db->dim, false), q->offsets, nullptr,
                    nullptr, ids, scores, flags, st);
  prof_end(st);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

size_t gift_query_exhaustive_static_bytes(const gift_views* db, const gift_queries* q,
                                          int32_t top_k, int32_t rescore_r) {
  return gift_query_exhaustive_workspace(db, q, top_k, rescore_r);
}

gift_status gift_query_exhaustive_static(const gift_views* db, const gift_queries* q,
                                         int32_t top_k, int32_t rescore_r, int32_t* ids,
                                         float* scores, int32_t* flags, void* stream) {
  gift_status s = check_views(db);
  if (s != GIFT_OK) return s;
  if ((s = check_queries(q, db->dim)) != GIFT_OK) return s;
  const size_t need = carve_exhaustive(nullptr, db, q, rescore_r > 0 ? rescore_r : 1).bytes;
  GIFT_CHECK(need <= (size_t)GIFT_STATIC_SCRATCH_BYTES, GIFT_ECAPACITY,
             "the batch needs %zu bytes of scratch; the static scratch holds %zu "
             "(use gift_query_exhaustive with a workspace)",
             need, (size_t)GIFT_STATIC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((s = static_scratch(&ws)) != GIFT_OK) return s;
  return gift_query_exhaustive(db, q, top_k, rescore_r, ids, scores, flags, ws,
                               (size_t)GIFT_STATIC_SCRATCH_BYTES, stream);
}

/* ------------------------------------------------------------ quantizer */
size_t gift_assign_workspace(int64_t n, int32_t dim, int32_t K, int32_t ma) {
  (void)ma;
  Carver c(nullptr);
  carve_assign(c, n, K, dim);
  return c.bytes();
}

gift_status gift_assign(const float* x, int64_t n, int32_t dim, const float* codebook, int32_t K,
                        int32_t ma, int32_t* words, int32_t* n_uncertified, void* ws,
                        size_t ws_bytes, void* stream) {
  gift_status s = check_codebook(codebook, K, ma, dim);
  if (s != GIFT_OK) return s;
  GIFT_CHECK(x && words && n >= 0, GIFT_EINVAL, "null input/output or n < 0");
  GIFT_CHECK(aligned(x, 16), GIFT_EINVAL, "input rows must be 16-byte aligned");
  const hipStream_t st = (hipStream_t)stream;
  Carver c(ws);
  AssignWs w = carve_assign(c, n, K, dim);
  GIFT_CHECK(ws != nullptr && ws_bytes >= c.bytes(), GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", c.bytes(), ws_bytes);
  int32_t* ovf = n_uncertified ? n_uncertified : w.overflow;
  launch_fill_i32(ovf, 1, 0, st);
  GIFT_LAUNCHED();
  prof_begin(P_ASSIGN, st);
  s = launch_assign(x, n, dim, codebook, K, ma, words, w.D, w.chunk, w.nhi, w.nlo, ovf, w.xs,
                    w.cbs, st);
  prof_end(st);
  return s;
}

/* ------------------------------------------------------------ codebook */
struct KmWs {
  float* cb2;
  int32_t* a2;
  int32_t* members;
  int64_t* moff;
  int32_t* changes;
  int64_t* idx;
  void* bucket;
  AssignWs as;
  size_t bytes;
};

static KmWs carve_km(void* base, int64_t n, int dim, int K) {
  Carver c(base);
  KmWs w{};
  w.cb2 = c.take<float>((size_t)K * dim);
  w.a2 = c.take<int32_t>((size_t)n);
  w.members = c.take<int32_t>((size_t)n);
  w.moff = c.take<int64_t>((size_t)K + 1);
  w.changes = c.take<int32_t>(1);
  w.idx = c.take<int64_t>((size_t)K);
  w.bucket = c.take<uint8_t>(bucket_sort_ws(n, K));
  w.as = carve_assign(c, n, K, dim);
  w.bytes = c.bytes();
  return w;
}

size_t gift_build_codebook_workspace(int64_t n, int32_t dim, int32_t K) {
  return carve_km(nullptr, n, dim, K).bytes;
}

gift_status gift_build_codebook(const float* train, int64_t n, int32_t dim, int32_t K,
                                const int64_t* init_idx, int32_t max_iter, float* codebook,
                                int32_t* assign, int32_t* iters_run, void* ws, size_t ws_bytes,
                                void* stream) {
  gift_status s = check_codebook(train, K, 1, dim);
  if (s != GIFT_OK) return s;
  GIFT_CHECK(train && init_idx && codebook && assign && n >= K && max_iter >= 0, GIFT_EINVAL,
             "bad arguments (need n >= K, non-null buffers)");
  GIFT_CHECK(n < ((int64_t)1 << 31), GIFT_ECAPACITY, "n too large");
  for (int k = 0; k < K; ++k)
    GIFT_CHECK(init_idx[k] >= 0 && init_idx[k] < n, GIFT_EINVAL, "init_idx[%d] out of range", k);
  const hipStream_t st = (hipStream_t)stream;
  KmWs w = carve_km(ws, n, dim, K);
  GIFT_CHECK(ws != nullptr && ws_bytes >= w.bytes, GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", w.bytes, ws_bytes);
  GIFT_HIP(hipMemcpyAsync(w.idx, init_idx, (size_t)K * 8, hipMemcpyHostToDevice, st));
  launch_gather_rows(train, w.idx, K, dim, codebook, st);
  GIFT_LAUNCHED();
  launch_fill_i32(w.as.overflow, 1, 0, st);
  s = launch_assign(train, n, dim, codebook, K, 1, assign, w.as.D, w.as.chunk, w.as.nhi,
                    w.as.nlo, w.as.overflow, w.as.xs, w.as.cbs, st);
  if (s != GIFT_OK) return s;
  float* cur = codebook;
  float* nxt = w.cb2;
  int32_t* a_cur = assign;
  int32_t* a_nxt = w.a2;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    s = launch_bucket_sort(a_cur, n, K, w.moff, 0, 1, 1, w.members, nullptr, w.bucket, st);
    if (s != GIFT_OK) return s;
    launch_centroids(train, dim, K, w.moff, w.members, cur, nxt, st);
    GIFT_LAUNCHED();
    s = launch_assign(train, n, dim, nxt, K, 1, a_nxt, w.as.D, w.as.chunk, w.as.nhi, w.as.nlo,
                      w.as.overflow, w.as.xs, w.as.cbs, st);
    if (s != GIFT_OK) return s;
    launch_fill_i32(w.changes, 1, 0, st);
    launch_count_changes(a_cur, a_nxt, n, w.changes, st);
    GIFT_LAUNCHED();
    int32_t changes = 0;
    GIFT_HIP(hipMemcpyAsync(&changes, w.changes, 4, hipMemcpyDeviceToHost, st));
    GIFT_HIP(hipStreamSynchronize(st));
    float* t = cur; cur = nxt; nxt = t;
    int32_t* ta = a_cur; a_cur = a_nxt; a_nxt = ta;
    if (changes == 0) break;
  }
  if (it > max_iter) it = max_iter;
  if (cur != codebook)
    GIFT_HIP(hipMemcpyAsync(codebook, cur, (size_t)K * dim * 4, hipMemcpyDeviceToDevice, st));
  if (a_cur != assign)
    GIFT_HIP(hipMemcpyAsync(assign, a_cur, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
  int32_t ovf = 0;
  GIFT_HIP(hipMemcpyAsync(&ovf, w.as.overflow, 4, hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipStreamSynchronize(st));
  if (iters_run) *iters_run = it;
  GIFT_CHECK(ovf == 0, GIFT_ECAPACITY, "%d assignments had more than 256 near-tied codewords", ovf);
  return GIFT_OK;
}

/* ------------------------------------------------------------ F-IF build */
size_t gift_build_fif_workspace(const gift_views* db, int32_t K, int32_t ma) {
  if (check_views(db) != GIFT_OK) return 0;
  const int64_t nv = db->n_shapes * db->n_views;
  Carver c(nullptr);
  carve_assign(c, nv, K, db->dim);
  c.take<uint8_t>(bucket_sort_ws(nv * ma, K));
  return c.bytes();
}

gift_status gift_build_fif(const gift_views* db, const float* codebook, int32_t K, int32_t ma,
                           int64_t* offsets, int32_t* entry_shape, int32_t* entry_view,
                           int32_t* view_words, void* ws, size_t ws_bytes, void* stream) {
  gift_status s = check_views(db);
  if (s != GIFT_OK) return s;
  if ((s = check_codebook(codebook, K, ma, db->dim)) != GIFT_OK) return s;
  GIFT_CHECK(db->master != nullptr, GIFT_EINVAL, "the quantizer needs float32 master views");
  GIFT_CHECK(offsets && entry_shape && entry_view && view_words, GIFT_EINVAL, "null outputs");
  const int64_t nv = db->n_shapes * db->n_views;
  GIFT_CHECK(nv * ma < ((int64_t)1 << 31), GIFT_ECAPACITY, "too many entries");
  const hipStream_t st = (hipStream_t)stream;
  Carver c(ws);
  AssignWs w = carve_assign(c, nv, K, db->dim);
  void* bucket = c.take<uint8_t>(bucket_sort_ws(nv * ma, K));
  GIFT_CHECK(ws != nullptr && ws_bytes >= c.bytes(), GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", c.bytes(), ws_bytes);
  launch_fill_i32(w.overflow, 1, 0, st);
  GIFT_LAUNCHED();
  s = launch_assign(db->master, nv, db->dim, codebook, K, ma, view_words, w.D, w.chunk, w.nhi,
                    w.nlo, w.overflow, w.xs, w.cbs, st);
  if (s != GIFT_OK) return s;
  s = launch_bucket_sort(view_words, nv * ma, K, offsets, 1, ma, db->n_views, entry_shape,
                         entry_view, bucket, st);
  if (s != GIFT_OK) return s;
  int32_t ovf = 0;
  GIFT_HIP(hipMemcpyAsync(&ovf, w.overflow, 4, hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipStreamSynchronize(st));
  GIFT_CHECK(ovf == 0, GIFT_ECAPACITY, "%d views had more than 256 near-tied codewords", ovf);
  return GIFT_OK;
}

/* ------------------------------------------------------------ F-IF query */
size_t gift_query_fif_workspace(const gift_views* db, const gift_fif* fif,
                                const gift_queries* q, int32_t top_k, int32_t rescore_r) {
  (void)top_k;
  if (check_views(db) != GIFT_OK || check_queries(q, db->dim) != GIFT_OK || fif == nullptr)
    return 0;
  return carve_fif(nullptr, db, fif, q, rescore_r > 0 ? rescore_r : 1).bytes;
}

gift_status gift_query_fif(const gift_views* db, const gift_fif* fif, const gift_queries* q,
                           int32_t top_k, int32_t rescore_r, int32_t* ids, float* scores,
                           int32_t* flags, void* ws, size_t ws_bytes, void* stream) {
  gift_status s = check_views(db);
  if (s != GIFT_OK) return s;
  if ((s = check_queries(q, db->dim)) != GIFT_OK) return s;
  if ((s = check_fif(fif, db)) != GIFT_OK) return s;
  GIFT_CHECK(ids && scores, GIFT_EINVAL, "null outputs");
  GIFT_CHECK(top_k >= 1 && top_k <= rescore_r && rescore_r <= 1024 &&
                 (int64_t)rescore_r <= db->n_shapes,
             GIFT_EINVAL, "need 1 <= top_k <= rescore_r <= min(1024, N)");
  GIFT_CHECK(db->master != nullptr, GIFT_EINVAL, "the exact rescore needs float32 master views");
  const hipStream_t st = (hipStream_t)stream;
  FifWs w = carve_fif(ws, db, fif, q, rescore_r);
  GIFT_CHECK(ws != nullptr && ws_bytes >= w.bytes, GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", w.bytes, ws_bytes);
  if ((s = fif_first_pass(db, fif, q, w, st)) != GIFT_OK) return s;
  prof_begin(P_SELECT, st);
  launch_select_top(w.S, db->n_shapes, q->n_queries, rescore_r, nullptr, w.cand, w.cand_s,
                    w.sel_tmp, st);
  prof_end(st);
  GIFT_LAUNCHED();
  prof_begin(P_RESCORE, st);
  launch_rescore(db->master, db->n_views, db->dim, q->views, q->offsets, q->n_queries,
                 q->total_views, w.cand, rescore_r, top_k, rescore_dot_err(db->dim), w.qwords,
                 fif->view_words, fif->ma, nullptr, w.cand_s, first_pass_err(db->dtype, db->dim, true),
                 w.rs, w.s_hi, w.s_lo, st);
  prof_end(st);
  GIFT_LAUNCHED();
  prof_begin(P_FINAL, st);
  launch_final_rank(w.cand, w.cand_s, w.s_hi, w.s_lo, q->n_queries, rescore_r, top_k,
                    db->n_shapes, first_pass_err(db->dtype, db->dim, true), q->offsets,
                    w.as.overflow, nullptr, ids, scores, flags, st);
  prof_end(st);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

size_t gift_score_fif_workspace(const gift_views* db, const gift_fif* fif,
                                const gift_queries* q) {
  if (check_views(db) != GIFT_OK || check_queries(q, db->dim) != GIFT_OK || fif == nullptr)
    return 0;
  return carve_fif(nullptr, db, fif, q, 0).bytes;
}

gift_status gift_score_fif(const gift_views* db, const gift_fif* fif, const gift_queries* q,
                           float* scores, int32_t* qwords, void* ws, size_t ws_bytes,
                           void* stream) {
  gift_status s = check_views(db);
  if (s != GIFT_OK) return s;
  if ((s = check_queries(q, db->dim)) != GIFT_OK) return s;
  if ((s = check_fif(fif, db)) != GIFT_OK) return s;
  GIFT_CHECK(scores != nullptr, GIFT_EINVAL, "null scores");
  const hipStream_t st = (hipStream_t)stream;
  FifWs w = carve_fif(ws, db, fif, q, 0);
  GIFT_CHECK(ws != nullptr && ws_bytes >= w.bytes, GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", w.bytes, ws_bytes);
  w.S = scores;
  if ((s = fif_first_pass(db, fif, q, w, st)) != GIFT_OK) return s;
  if (qwords)
    GIFT_HIP(hipMemcpyAsync(qwords, w.qwords, (size_t)q->total_views * 4,
                            hipMemcpyDeviceToDevice, st));
  return GIFT_OK;
}

/* ------------------------------------------------------------ tuning */
gift_status gift_copy_async(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes == 0) return GIFT_OK;
  GIFT_CHECK(dst != nullptr && src != nullptr, GIFT_EINVAL, "null buffer");
  GIFT_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, static_cast<hipStream_t>(stream)));
  return GIFT_OK;
}

gift_status gift_set_score_tuning(int32_t dtype, int32_t tile, int32_t group) {
  return set_score_tuning(dtype, tile, group);
}

gift_status gift_get_score_tuning(int32_t dtype, int32_t* tile, int32_t* group) {
  GIFT_CHECK(dtype >= 0 && dtype <= 2 && tile && group, GIFT_EINVAL, "bad arguments");
  get_score_tuning(dtype, tile, group);
  return GIFT_OK;
}

gift_status gift_autotune_score(const gift_views* db, const gift_queries* q, const int32_t* tiles,
                                int32_t n_tiles, const int32_t* groups, int32_t n_groups,
                                int32_t reps, float* ms_out, int32_t* best_tile,
                                int32_t* best_group, void* ws, size_t ws_bytes, void* stream) {
  gift_status s = check_views(db);
  if (s != GIFT_OK) return s;
  if ((s = check_queries(q, db->dim)) != GIFT_OK) return s;
  GIFT_CHECK(tiles && groups && n_tiles >= 1 && n_groups >= 1 && reps >= 1 && best_tile &&
                 best_group, GIFT_EINVAL, "bad arguments");
  const hipStream_t st = (hipStream_t)stream;
  ExhaustiveWs w = carve_exhaustive(ws, db, q, 0);
  GIFT_CHECK(ws != nullptr && ws_bytes >= w.bytes, GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", w.bytes, ws_bytes);
  int keep_tile = 0, keep_group = 8;
  get_score_tuning(db->dtype, &keep_tile, &keep_group);
  const void* qv = q->views;
  const void* qs = nullptr;
  if (db->dtype != GIFT_F32) {
    launch_quantize(q->views, q->total_views, db->dim, db->dtype, w.qcodes, w.qscale, st);
    GIFT_LAUNCHED();
    qv = w.qcodes;
    qs = w.qscale;
  }
  hipEvent_t e0, e1;
  GIFT_HIP(hipEventCreate(&e0));
  GIFT_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  *best_tile = keep_tile;
  *best_group = keep_group;
  for (int a = 0; a < n_tiles; ++a)
    for (int g = 0; g < n_groups; ++g) {
      s = set_score_tuning(db->dtype, tiles[a], groups[g]);
      if (s == GIFT_OK) s = launch_score_tiles(db, qv, qs, q->total_views, w.mbuf, q->total_views, st);
      if (s == GIFT_OK) GIFT_HIP(hipEventRecord(e0, st));
      for (int r = 0; s == GIFT_OK && r < reps; ++r)
        s = launch_score_tiles(db, qv, qs, q->total_views, w.mbuf, q->total_views, st);
      float ms = 0.f;
      if (s == GIFT_OK) {
        GIFT_HIP(hipEventRecord(e1, st));
        GIFT_HIP(hipEventSynchronize(e1));
        GIFT_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms /= reps;
      }
      if (s != GIFT_OK) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        set_score_tuning(db->dtype, keep_tile, keep_group);
        return s;
      }
      if (ms_out) ms_out[a * n_groups + g] = ms;
      if (ms < best) {
        best = ms;
        *best_tile = tiles[a];
        *best_group = groups[g];
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return set_score_tuning(db->dtype, *best_tile, *best_group);
}

/* ------------------------------------------------------------ S-IF */
size_t gift_build_sif_workspace(int64_t n_shapes) {
  Carver c(nullptr);
  c.take<unsigned long long>((size_t)n_shapes);
  c.take<unsigned long long>((size_t)n_shapes);
  return c.bytes();
}

gift_status gift_build_sif(int64_t n_shapes, int32_t k1, const int32_t* nbr_ids,
                           const float* nbr_scores, float* l1, int64_t* post_off,
                           int32_t* post_id, float* post_val, void* ws, size_t ws_bytes,
                           void* stream) {
  GIFT_CHECK(n_shapes >= 1 && n_shapes < ((int64_t)1 << 31), GIFT_EINVAL, "n_shapes out of range");
  GIFT_CHECK(k1 >= 1 && k1 <= 256, GIFT_EINVAL, "k1 must be in 1..256");
  GIFT_CHECK(n_shapes * k1 < ((int64_t)1 << 31), GIFT_ECAPACITY, "n_shapes * k1 too large");
  GIFT_CHECK(nbr_ids && nbr_scores && l1 && post_off && post_id && post_val, GIFT_EINVAL,
             "null pointer");
  Carver c(ws);
  auto* cnt = c.take<unsigned long long>((size_t)n_shapes);
  auto* fill = c.take<unsigned long long>((size_t)n_shapes);
  GIFT_CHECK(ws != nullptr && ws_bytes >= c.bytes(), GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", c.bytes(), ws_bytes);
  launch_build_sif(nbr_ids, nbr_scores, n_shapes, k1, l1, post_off, post_id, post_val, cnt,
                   fill, (hipStream_t)stream);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

gift_status gift_augment_neighbours(int64_t n_shapes, int32_t k1, const int32_t* nbr_ids,
                                   const float* nbr_scores, int32_t n_rows,
                                   const int32_t* members, int32_t k2, const int32_t* own_ids,
                                   const float* own_scores, int32_t k_own, int32_t* out_ids,
                                   float* out_scores, int32_t k_out, int32_t* n_members,
                                   void* stream) {
  GIFT_CHECK(n_shapes >= 1 && n_shapes < ((int64_t)1 << 31), GIFT_EINVAL, "n_shapes out of range");
  GIFT_CHECK(k1 >= 1 && k2 >= 1 && n_rows >= 0, GIFT_EINVAL, "bad sizes");
  GIFT_CHECK(own_ids == nullptr || (own_scores != nullptr && k_own >= 1), GIFT_EINVAL,
             "own row needs scores and k_own >= 1");
  const int total = k2 * k1 + (own_ids ? k_own : 0);
  GIFT_CHECK(total <= 1024, GIFT_EUNSUPPORTED, "k2 * k1 + k_own must be <= 1024");
  GIFT_CHECK(k_out >= 1, GIFT_EINVAL, "k_out must be >= 1");
  GIFT_CHECK(nbr_ids && nbr_scores && members && out_ids && out_scores, GIFT_EINVAL,
             "null pointer");
  launch_augment(nbr_ids, nbr_scores, n_shapes, k1, members, k2, own_ids, own_scores, k_own,
                 n_rows, out_ids, out_scores, k_out, n_members, (hipStream_t)stream);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

gift_status gift_fuse_activations(int32_t n_rows, const int32_t* ids1, const float* scores1,
                                 int32_t k_a, const int32_t* ids2, const float* scores2,
                                 int32_t k_b, float alpha, int32_t* out_ids, float* out_scores,
                                 int32_t k_out, void* stream) {
  GIFT_CHECK(n_rows >= 0 && k_a >= 1 && k_b >= 1 && k_a + k_b <= 1024 && k_out >= 1,
             GIFT_EINVAL, "bad sizes (k_a + k_b <= 1024)");
  GIFT_CHECK(alpha > 0.f, GIFT_EINVAL, "alpha must be > 0");
  GIFT_CHECK(ids1 && scores1 && ids2 && scores2 && out_ids && out_scores, GIFT_EINVAL,
             "null pointer");
  launch_fuse(ids1, scores1, k_a, ids2, scores2, k_b, alpha, n_rows, out_ids, out_scores, k_out,
              (hipStream_t)stream);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

gift_status gift_fuse_self(int32_t n_rows, const float* self1, const int32_t* n1,
                           const float* self2, const int32_t* n2, float alpha, float* out,
                           void* stream) {
  GIFT_CHECK(n_rows >= 0, GIFT_EINVAL, "n_rows < 0");
  GIFT_CHECK(alpha > 0.f, GIFT_EINVAL, "alpha must be > 0");
  GIFT_CHECK(n_rows == 0 || (self1 && n1 && self2 && n2 && out), GIFT_EINVAL, "null pointer");
  launch_fuse_self(self1, n1, self2, n2, alpha, n_rows, out, (hipStream_t)stream);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

gift_status gift_rerank_sif(int64_t n_shapes, const float* l1, const int64_t* post_off,
                            const int32_t* post_id, const float* post_val, int32_t n_queries,
                            int32_t k1, const int32_t* q_ids, const float* q_scores,
                            const float* q_self, int32_t top_k, int32_t* ids, float* scores,
                            int32_t* flags, void* stream) {
  GIFT_CHECK(n_shapes >= 1 && n_shapes < ((int64_t)1 << 31), GIFT_EINVAL, "n_shapes out of range");
  GIFT_CHECK(k1 >= 1 && k1 <= 256, GIFT_EINVAL, "k1 must be in 1..256");
  GIFT_CHECK(top_k >= 1 && top_k <= n_shapes && top_k <= 1024, GIFT_EINVAL,
             "need 1 <= top_k <= min(n_shapes, 1024)");
  GIFT_CHECK(n_queries >= 0, GIFT_EINVAL, "n_queries < 0");
  GIFT_CHECK(l1 && post_off && post_id && post_val && q_ids && q_scores && ids && scores,
             GIFT_EINVAL, "null pointer");
  const hipStream_t st = (hipStream_t)stream;
  prof_begin(P_RERANK, st);
  launch_rerank_sif(l1, post_off, post_id, post_val, n_shapes, q_ids, q_scores, q_self,
                    n_queries, k1, top_k, ids, scores, flags, st);
  prof_end(st);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

}  // extern "C"
