// Batch plans: the whole F-IF query path of a ragged batch (Eq. 4 first
// pass in one persistent kernel, then selection, exact rescore and final
// ranking) captured once into a HIP graph and replayed per batch.
#include <string.h>

#include "kernels.h"

namespace gift {

struct PlanWs {
  float* nhi;
  float* nlo;
  int64_t* tcount;
  int64_t* tile_off;
  int32_t* tile_word;
  int32_t* act_off;
  int32_t* act_tile;
  int32_t* desc;
  uint8_t* qcodes;
  void* qscale;
  uint8_t* qsplit;   // query views split into BF16 parts (codeword GEMM)
  uint8_t* cbsplit;  // codebook split into BF16 parts
  float* D;
  int32_t* qwords;
  int32_t* counts;
  int64_t* goff;
  int32_t* fillc;
  int32_t* gitems;
  uint32_t* mbuf;
  float* S;
  int32_t* overflow;
  unsigned long long* ctrl;
  unsigned long long* phase_ticks;
  int32_t* cand;
  float* cand_s;
  void* sel_tmp;  // chunk winners of the top-r selection
  float* s_hi;
  float* s_lo;
  RescoreScratch rs;  // rescore masks [r][Vmax], approximate scores, top-k marks
  size_t bytes;
};

static PlanWs carve_plan(void* base, const gift_views* db, const gift_fif* f, int Bmax,
                         int64_t Vmax, int r, int tile_len) {
  Carver c(base);
  PlanWs w{};
  w.nhi = c.take<float>((size_t)f->K);
  w.nlo = c.take<float>((size_t)f->K);
  w.tcount = c.take<int64_t>((size_t)f->K);
  w.tile_off = c.take<int64_t>((size_t)f->K + 1);
  // list tiles: at most n_entries / tile_len + K of them
  const size_t max_tiles = (size_t)(f->n_entries / tile_len + f->K + 1);
  w.tile_word = c.take<int32_t>(max_tiles);
  w.act_off = c.take<int32_t>((size_t)f->K);
  w.act_tile = c.take<int32_t>(max_tiles);
  w.desc = c.take<int32_t>(4);
  if (db->dtype != GIFT_F32) {
    w.qcodes = c.take<uint8_t>((size_t)Vmax * row_bytes_of(db->dtype, db->dim));
    // per-view float32 scales, or E8M0 rows of dim / 32 bytes (MX)
    w.qscale = c.take<uint8_t>(is_mx(db->dtype) ? (size_t)Vmax * (db->dim / 32)
                                                : (size_t)Vmax * sizeof(float));
  }
  w.qsplit = c.take<uint8_t>((size_t)Vmax * db->dim * 4);
  w.cbsplit = c.take<uint8_t>((size_t)f->K * db->dim * 4);
  w.D = c.take<float>((size_t)Vmax * f->K);
  w.qwords = c.take<int32_t>((size_t)Vmax);
  w.counts = c.take<int32_t>((size_t)f->K);
  w.goff = c.take<int64_t>((size_t)f->K + 1);
  w.fillc = c.take<int32_t>((size_t)f->K);
  w.gitems = c.take<int32_t>((size_t)Vmax);
  w.mbuf = c.take<uint32_t>((size_t)db->n_shapes * Vmax);
  w.S = c.take<float>((size_t)Bmax * db->n_shapes);
  w.overflow = c.take<int32_t>(1);
  w.ctrl = c.take<unsigned long long>(BATCH_CTRL_WORDS);
  w.phase_ticks = c.take<unsigned long long>(2 * BP_END + 1);
  w.cand = c.take<int32_t>((size_t)Bmax * r);
  w.cand_s = c.take<float>((size_t)Bmax * r);
  w.sel_tmp = c.take<uint8_t>(select_top_ws(db->n_shapes, Bmax, r));
  w.s_hi = c.take<float>((size_t)Bmax * r);
  w.s_lo = c.take<float>((size_t)Bmax * r);
  w.rs = take_rescore(c, Bmax, r, Vmax);
  // partial tiles of the split approximate phase (used when the plan's
  // queries have at most 64 views; see gift_fif_plan_create)
  const size_t pf = rescore_split_floats(Bmax, r);
  if (pf != 0) w.rs.part = c.take<float>(pf);
  w.bytes = c.bytes();
  return w;
}

}  // namespace gift

struct gift_fif_plan {
  gift::BatchArgs args;
  gift::PlanWs ws;
  gift_views db;
  int Bmax, max_m, top_k, r;
  int64_t Vmax;
  int grid;
  const float* qviews;
  int32_t* qoff;
  int32_t* ids;
  float* scores;
  int32_t* flags;
  const int32_t* view_words;
  int ma;
  hipGraph_t graph;
  hipGraphExec_t exec;
  int clock_khz;
};

namespace gift {

static gift_status enqueue_plan(gift_fif_plan* p, hipStream_t st) {
  launch_batch_reset(p->args, st);
  GIFT_LAUNCHED();
  if (p->args.ext_gemm) {
    const gift_status s0 = launch_batch_pre(p->args, p->db.dtype, st);
    if (s0 != GIFT_OK) return s0;
  }
  gift_status s = launch_fif_batch(p->args, p->db.dtype, p->grid, st);
  if (s != GIFT_OK) return s;
  // query slots past the batch (desc[0]) are skipped by every ranking kernel
  const int32_t* active = p->ws.desc;
  launch_select_top(p->ws.S, p->db.n_shapes, p->Bmax, p->r, active, p->ws.cand, p->ws.cand_s,
                    p->ws.sel_tmp, st);
  GIFT_LAUNCHED();
  launch_rescore(p->db.master, p->db.n_views, p->db.dim, p->qviews, p->qoff, p->Bmax, p->Vmax,
                 p->ws.cand, p->r, p->top_k, rescore_dot_error(p->db.dim), p->ws.qwords,
                 p->view_words, p->ma, active, p->ws.cand_s,
                 first_pass_error(p->db.dtype, p->db.dim, true), p->ws.rs, p->ws.s_hi, p->ws.s_lo, st);
  GIFT_LAUNCHED();
  launch_final_rank(p->ws.cand, p->ws.cand_s, p->ws.s_hi, p->ws.s_lo, p->Bmax, p->r, p->top_k,
                    p->db.n_shapes, first_pass_error(p->db.dtype, p->db.dim, true), p->qoff,
                    p->ws.overflow, active, p->ids, p->scores, p->flags, st);
  GIFT_LAUNCHED();
  return GIFT_OK;
}

}  // namespace gift

// The tuning a plan runs with: the given one, or the defaults (2 blocks per
// CU, 128-entry list tiles, narrow tiles for groups of up to 32 views, the
// codeword GEMM placed by capacity).
static gift_plan_tuning plan_tuning(const gift_plan_tuning* t) {
  if (t != nullptr) return *t;
  gift_plan_tuning d{};
  d.blocks_per_cu = 2;
  d.list_tile = 128;
  d.narrow_max = 32;
  d.gemm = 0;
  return d;
}

static bool tuning_ok(const gift_plan_tuning& t) {
  return (t.blocks_per_cu == 1 || t.blocks_per_cu == 2) && t.list_tile >= 32 &&
         t.list_tile <= 128 && t.list_tile % 32 == 0 &&
         (t.narrow_max == 0 || t.narrow_max == 16 || t.narrow_max == 32) && t.gemm >= 0 &&
         t.gemm <= 2;
}

// Large batches take the separate 256 x 256 GEMM kernel (about half the
// BF16 MFMA peak against a third for the persistent kernel's 128 x 128 dot
// items); small ones keep the dot items, which spread one query's few row
// tiles over more blocks.
constexpr int64_t PLAN_EXT_GEMM_VIEWS = 16384;

using namespace gift;

extern "C" {

size_t gift_fif_plan_workspace(const gift_views* db, const gift_fif* fif, int32_t max_queries,
                               int64_t max_views, int32_t top_k, int32_t rescore_r,
                               const gift_plan_tuning* tuning) {
  (void)top_k;
  const gift_plan_tuning t = plan_tuning(tuning);
  if (db == nullptr || fif == nullptr || max_queries < 1 || max_views < 1 || rescore_r < 1 ||
      !tuning_ok(t))
    return 0;
  return carve_plan(nullptr, db, fif, max_queries, max_views, rescore_r, t.list_tile).bytes;
}

gift_status gift_fif_plan_create(const gift_views* db, const gift_fif* fif, int32_t max_queries,
                                 int64_t max_views, int32_t max_views_per_query, int32_t top_k,
                                 int32_t rescore_r, const float* q_views, int32_t* q_offsets,
                                 int32_t* ids, float* scores, int32_t* flags,
                                 const gift_plan_tuning* tuning, void* ws, size_t ws_bytes,
                                 void* stream, gift_fif_plan** plan) {
  GIFT_CHECK(plan != nullptr, GIFT_EINVAL, "null plan pointer");
  *plan = nullptr;
  GIFT_CHECK(db && fif && db->data && db->master && fif->codebook && fif->offsets &&
                 fif->entry_shape && fif->entry_view && fif->view_words,
             GIFT_EINVAL, "incomplete database or index (the plan needs float32 master views)");
  GIFT_CHECK(db->n_views >= 1 && db->n_views <= 64 && db->dim >= 32 && db->dim % 32 == 0,
             GIFT_EUNSUPPORTED, "n_views must be 1..64 and dim a multiple of 32");
  GIFT_CHECK(db->dtype == GIFT_F32 || db->scale != nullptr, GIFT_EINVAL, "missing scales");
  GIFT_CHECK(db->dtype != GIFT_MXFP8 || db->dim % 128 == 0, GIFT_EUNSUPPORTED,
             "MXFP8 storage needs dim a multiple of 128");
  GIFT_CHECK(db->dtype != GIFT_MXFP4 || db->dim % 256 == 0, GIFT_EUNSUPPORTED,
             "MXFP4 storage needs dim a multiple of 256");
  GIFT_CHECK(fif->K >= 1 && fif->K <= 16384 && fif->ma >= 1 && fif->ma <= 8, GIFT_EUNSUPPORTED,
             "K must be 1..16384 and ma 1..8");
  GIFT_CHECK(fif->n_entries == (int64_t)fif->ma * db->n_shapes * db->n_views, GIFT_EINVAL,
             "n_entries must be ma * n_shapes * n_views");
  const gift_plan_tuning tune = plan_tuning(tuning);
  GIFT_CHECK(tuning_ok(tune), GIFT_EINVAL,
             "tuning: blocks_per_cu 1 or 2, list_tile 32..128 in steps of 32, narrow_max 0, "
             "16 or 32, gemm 0..2");
  GIFT_CHECK(fif->n_entries / tune.list_tile + fif->K + 1 < ((int64_t)1 << 31), GIFT_ECAPACITY,
             "too many list tiles");
  GIFT_CHECK(max_queries >= 1 && max_views >= 1 && max_views < ((int64_t)1 << 31) &&
                 max_views_per_query >= 1,
             GIFT_EINVAL, "bad capacities");
  GIFT_CHECK(top_k >= 1 && top_k <= rescore_r && rescore_r <= 1024 &&
                 (int64_t)rescore_r <= db->n_shapes,
             GIFT_EINVAL, "need 1 <= top_k <= rescore_r <= min(1024, N)");
  GIFT_CHECK(q_views && q_offsets && ids && scores, GIFT_EINVAL, "null batch buffers");
  GIFT_CHECK((reinterpret_cast<uintptr_t>(q_views) & 15) == 0 &&
                 (reinterpret_cast<uintptr_t>(db->data) & 15) == 0 &&
                 (reinterpret_cast<uintptr_t>(db->master) & 15) == 0,
             GIFT_EINVAL, "views must be 16-byte aligned");
  const hipStream_t st = (hipStream_t)stream;
  PlanWs w = carve_plan(ws, db, fif, max_queries, max_views, rescore_r, tune.list_tile);
  GIFT_CHECK(ws != nullptr && ws_bytes >= w.bytes, GIFT_EWORKSPACE,
             "workspace needs %zu bytes, got %zu", w.bytes, ws_bytes);

  // When the plan's queries have at most 64 views, a batch of at most
  // RESCORE_SPLIT_ITEMS work items (4 candidates of one query each: one
  // query at r = 256, four at r = 64) splits the approximate rescore phase
  // over K, 4 blocks per item of 2+ K-tiles each, so its K loop does not
  // run on a handful of blocks; larger batches take the one-block-per-item
  // kernel (the choice is made per run from the batch size)
  w.rs.n_split = (w.rs.part != nullptr && max_views_per_query <= 64 && db->dim / 32 >= 2 * RESCORE_SPLIT)
                     ? RESCORE_SPLIT
                     : 0;
  auto* p = new gift_fif_plan();
  p->ws = w;
  p->db = *db;
  p->Bmax = max_queries;
  p->Vmax = max_views;
  p->max_m = max_views_per_query;
  p->top_k = top_k;
  p->r = rescore_r;
  p->qviews = q_views;
  p->qoff = q_offsets;
  p->ids = ids;
  p->scores = scores;
  p->flags = flags;
  p->view_words = fif->view_words;
  p->ma = fif->ma;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    delete p;
    return fail(GIFT_EHIP, "cannot query the device");
  }
  p->grid = n_cu * tune.blocks_per_cu;
  int clock_khz = 0;
  if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      clock_khz <= 0) {
    delete p;
    return fail(GIFT_EHIP, "cannot query the wall-clock rate");
  }

  // once per plan: codebook norms, split codebook and list-tile offsets
  gift_status s = launch_norms(fif->codebook, fif->K, db->dim, w.nhi, w.nlo, st);
  if (s == GIFT_OK) {
    launch_split_rows(fif->codebook, fif->K, db->dim, w.cbsplit, st);
    if (hipGetLastError() != hipSuccess) s = fail(GIFT_EHIP, "codebook split launch failed");
  }
  if (s == GIFT_OK)
    s = launch_list_tiles(fif->offsets, fif->K, tune.list_tile, w.tcount, w.tile_off, st);
  if (s == GIFT_OK) {
    launch_tile_word(w.tile_off, fif->K, w.tile_word, st);
    if (hipGetLastError() != hipSuccess) s = fail(GIFT_EHIP, "tile map launch failed");
  }
  if (s != GIFT_OK) {
    delete p;
    return s;
  }

  BatchArgs& a = p->args;
  memset(&a, 0, sizeof(a));
  a.db = static_cast<const uint8_t*>(db->data);
  a.db_scale = db->scale;
  a.n_views = db->n_views;
  a.row_bytes = (int)row_bytes_of(db->dtype, db->dim);
  a.n_shapes = db->n_shapes;
  a.cb = fif->codebook;
  a.nhi = w.nhi;
  a.nlo = w.nlo;
  a.K = fif->K;
  a.dim = db->dim;
  a.loff = fif->offsets;
  a.ent_shape = fif->entry_shape;
  a.ent_view = fif->entry_view;
  a.tile_off = w.tile_off;
  a.tile_word = w.tile_word;
  a.qviews = q_views;
  a.qsplit = w.qsplit;
  a.cbsplit = w.cbsplit;
  a.qoff = q_offsets;
  a.Bmax = max_queries;
  a.Vmax = max_views;
  a.desc = w.desc;
  a.qcodes = w.qcodes;
  a.qscale = w.qscale;
  a.D = w.D;
  a.qwords = w.qwords;
  a.counts = w.counts;
  a.goff = w.goff;
  a.fillc = w.fillc;
  a.gitems = w.gitems;
  a.act_off = w.act_off;
  a.act_tile = w.act_tile;
  a.mbuf = w.mbuf;
  a.S = w.S;
  a.overflow = w.overflow;
  a.ctrl = w.ctrl;
  a.phase_ticks = w.phase_ticks;
  a.gamma2 = assign_gamma2(db->dim);
  a.wait_ticks = (int64_t)clock_khz * 1000 * 5;  // five seconds per phase wait
  p->clock_khz = clock_khz;
  a.gemm_col_tiles = (fif->K + 127) / 128;
  a.tile_len = tune.list_tile;
  a.narrow_max = tune.narrow_max;
  a.ext_gemm = tune.gemm == 2 || (tune.gemm == 0 && max_views >= PLAN_EXT_GEMM_VIEWS) ? 1 : 0;

  // an empty batch run eagerly once (sets kernel attributes, checks launches)
  {
    const int32_t zero[2] = {0, 0};
    if (hipMemcpyAsync(w.desc, zero, sizeof(zero), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(q_offsets, zero, 4, hipMemcpyHostToDevice, st) != hipSuccess) {
      delete p;
      return fail(GIFT_EHIP, "plan initialisation copy failed");
    }
    s = enqueue_plan(p, st);
    if (s == GIFT_OK && hipStreamSynchronize(st) != hipSuccess)
      s = fail(GIFT_EHIP, "plan warm-up failed");
    if (s != GIFT_OK) {
      delete p;
      return s;
    }
  }

  // capture the batch into a graph
  hipStreamCaptureStatus cs;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
    delete p;
    return fail(GIFT_EINVAL, "the plan stream must not be capturing");
  }
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    delete p;
    return fail(GIFT_EHIP, "hipStreamBeginCapture failed");
  }
  s = enqueue_plan(p, st);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(st, &g);
  if (s != GIFT_OK || ec != hipSuccess || g == nullptr) {
    if (g) (void)hipGraphDestroy(g);
    delete p;
    return s != GIFT_OK ? s : fail(GIFT_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
  }
  p->graph = g;
  if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    delete p;
    return fail(GIFT_EHIP, "graph instantiation failed");
  }
  *plan = p;
  return GIFT_OK;
}

gift_status gift_fif_plan_run(gift_fif_plan* p, int32_t n_queries, int64_t n_views,
                              void* stream) {
  GIFT_CHECK(p != nullptr, GIFT_EINVAL, "null plan");
  GIFT_CHECK(n_queries >= 0 && n_queries <= p->Bmax && n_views >= 0 && n_views <= p->Vmax,
             GIFT_ECAPACITY, "batch of %d queries / %lld views exceeds the plan (%d / %lld)",
             n_queries, (long long)n_views, p->Bmax, (long long)p->Vmax);
  const hipStream_t st = (hipStream_t)stream;
  const int32_t desc[2] = {n_queries, (int32_t)n_views};
  // pageable source: the runtime stages it before returning, so `desc` may go
  GIFT_HIP(hipMemcpyAsync(p->ws.desc, desc, sizeof(desc), hipMemcpyHostToDevice, st));
  GIFT_HIP(hipGraphLaunch(p->exec, st));
  return GIFT_OK;
}

gift_status gift_fif_plan_serve(gift_fif_plan* p, const float* host_views,
                                const int32_t* host_offsets, int32_t n_queries, int64_t n_views,
                                int64_t n_shapes, const float* l1, const int64_t* post_off,
                                const int32_t* post_id, const float* post_val,
                                const float* q_self, int32_t top_k, int32_t* rr_ids,
                                float* rr_scores, int32_t* rr_flags, int32_t* host_ids,
                                float* host_scores, int32_t* host_flags, void* stream) {
  GIFT_CHECK(p != nullptr && host_views != nullptr && host_offsets != nullptr &&
                 host_ids != nullptr && host_scores != nullptr,
             GIFT_EINVAL, "null plan or host buffer");
  GIFT_CHECK(n_queries >= 0 && n_queries <= p->Bmax && n_views >= 0 && n_views <= p->Vmax,
             GIFT_ECAPACITY, "batch of %d queries / %lld views exceeds the plan (%d / %lld)",
             n_queries, (long long)n_views, p->Bmax, (long long)p->Vmax);
  const bool rerank = l1 != nullptr;
  GIFT_CHECK(!rerank || (post_off && post_id && post_val && rr_ids && rr_scores && rr_flags &&
                         host_flags && top_k >= 1 && n_shapes >= 1),
             GIFT_EINVAL, "incomplete S-IF re-rank arguments");
  if (n_queries == 0) return GIFT_OK;
  const hipStream_t st = (hipStream_t)stream;
  GIFT_HIP(hipMemcpyAsync(const_cast<float*>(p->qviews), host_views,
                          (size_t)n_views * p->db.dim * sizeof(float), hipMemcpyHostToDevice, st));
  GIFT_HIP(hipMemcpyAsync(p->qoff, host_offsets, (size_t)(n_queries + 1) * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
  const gift_status s = gift_fif_plan_run(p, n_queries, n_views, stream);
  if (s != GIFT_OK) return s;
  const int32_t* ids = p->ids;
  const float* sc = p->scores;
  const int32_t* fl = p->flags;
  int32_t k = p->top_k;
  if (rerank) {
    const gift_status r = gift_rerank_sif(n_shapes, l1, post_off, post_id, post_val, n_queries,
                                          p->top_k, p->ids, p->scores, q_self, top_k, rr_ids,
                                          rr_scores, rr_flags, stream);
    if (r != GIFT_OK) return r;
    ids = rr_ids;
    sc = rr_scores;
    fl = rr_flags;
    k = top_k;
  }
  const size_t n_out = (size_t)n_queries * k;
  GIFT_HIP(hipMemcpyAsync(host_ids, ids, n_out * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  GIFT_HIP(hipMemcpyAsync(host_scores, sc, n_out * sizeof(float), hipMemcpyDeviceToHost, st));
  if (host_flags != nullptr && fl != nullptr)
    GIFT_HIP(hipMemcpyAsync(host_flags, fl, (size_t)n_queries * sizeof(int32_t),
                            hipMemcpyDeviceToHost, st));
  return GIFT_OK;
}

gift_status gift_fif_plan_run_eager(gift_fif_plan* p, int32_t n_queries, int64_t n_views,
                                    void* stream) {
  GIFT_CHECK(p != nullptr, GIFT_EINVAL, "null plan");
  GIFT_CHECK(n_queries >= 0 && n_queries <= p->Bmax && n_views >= 0 && n_views <= p->Vmax,
             GIFT_ECAPACITY, "batch exceeds the plan");
  const hipStream_t st = (hipStream_t)stream;
  const int32_t desc[2] = {n_queries, (int32_t)n_views};
  GIFT_HIP(hipMemcpyAsync(p->ws.desc, desc, sizeof(desc), hipMemcpyHostToDevice, st));
  return enqueue_plan(p, st);
}

gift_status gift_fif_plan_first_pass(gift_fif_plan* p, int32_t n_queries, float* out,
                                     void* stream) {
  GIFT_CHECK(p != nullptr && out != nullptr, GIFT_EINVAL, "null argument");
  GIFT_CHECK(n_queries >= 0 && n_queries <= p->Bmax, GIFT_EINVAL, "n_queries out of range");
  GIFT_HIP(hipMemcpyAsync(out, p->ws.S, (size_t)n_queries * p->db.n_shapes * sizeof(float),
                          hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return GIFT_OK;
}

gift_status gift_fif_plan_error(gift_fif_plan* p, int32_t* err, void* stream) {
  GIFT_CHECK(p != nullptr && err != nullptr, GIFT_EINVAL, "null argument");
  unsigned long long e = 0;
  GIFT_HIP(hipMemcpyAsync(&e, p->ws.ctrl + 2, 8, hipMemcpyDeviceToHost, (hipStream_t)stream));
  GIFT_HIP(hipStreamSynchronize((hipStream_t)stream));
  *err = (int32_t)e;
  return GIFT_OK;
}

gift_status gift_fif_plan_phase_us(gift_fif_plan* p, double* out, void* stream) {
  GIFT_CHECK(p != nullptr && out != nullptr, GIFT_EINVAL, "null argument");
  unsigned long long t[BP_END];
  GIFT_HIP(hipMemcpyAsync(t, p->ws.phase_ticks, sizeof(t), hipMemcpyDeviceToHost,
                          (hipStream_t)stream));
  GIFT_HIP(hipStreamSynchronize((hipStream_t)stream));
  for (int i = 0; i < BP_END; ++i) out[i] = (double)t[i] * 1000.0 / (double)p->clock_khz;
  return GIFT_OK;
}

gift_status gift_fif_plan_phase_end_us(gift_fif_plan* p, double* out, void* stream) {
  GIFT_CHECK(p != nullptr && out != nullptr, GIFT_EINVAL, "null argument");
  unsigned long long t[2 * BP_END + 1];
  GIFT_HIP(hipMemcpyAsync(t, p->ws.phase_ticks, sizeof(t), hipMemcpyDeviceToHost,
                          (hipStream_t)stream));
  GIFT_HIP(hipStreamSynchronize((hipStream_t)stream));
  const unsigned long long t0 = t[2 * BP_END];
  for (int i = 0; i < BP_END; ++i) {
    const unsigned long long e = t[BP_END + i];
    out[i] = e > t0 ? (double)(e - t0) * 1000.0 / (double)p->clock_khz : 0.0;
  }
  return GIFT_OK;
}

gift_status gift_fif_plan_destroy(gift_fif_plan* p) {
  if (p == nullptr) return GIFT_OK;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  delete p;
  return GIFT_OK;
}

}  // extern "C"
