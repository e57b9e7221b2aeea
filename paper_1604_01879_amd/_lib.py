"""ctypes binding of libgift.so (argument marshalling only).

Every computation runs in the HIP kernels behind the C ABI declared in
include/gift.h.  torch tensors supply device memory and the current HIP
stream.  If the shared library is missing, importing this module raises: there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgift.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -m paper_1604_01879_amd.build`")
_lib = C.CDLL(LIB_PATH)

# status codes and storage formats (include/gift.h)
OK, EINVAL, EWORKSPACE, EUNSUPPORTED, EHIP, ECAPACITY = 0, -1, -2, -3, -4, -5
F32, BF16, FP8E4M3, MXFP8, MXFP4 = 0, 1, 2, 3, 4
_DT_TORCH = {F32: torch.float32, BF16: torch.uint16, FP8E4M3: torch.uint8, MXFP8: torch.uint8,
             MXFP4: torch.uint8}


class GiftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gift status {status}: {msg}")
        self.status = status


class gift_views(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("n_views", C.c_int32),
                ("n_shapes", C.c_int64), ("dim", C.c_int32), ("_pad", C.c_int32),
                ("scale", C.c_void_p), ("master", C.c_void_p)]


class gift_queries(C.Structure):
    _fields_ = [("views", C.c_void_p), ("offsets", C.c_void_p), ("n_queries", C.c_int32),
                ("max_views", C.c_int32), ("total_views", C.c_int64)]


class gift_fif(C.Structure):
    _fields_ = [("codebook", C.c_void_p), ("K", C.c_int32), ("ma", C.c_int32),
                ("n_entries", C.c_int64), ("offsets", C.c_void_p), ("entry_shape", C.c_void_p),
                ("entry_view", C.c_void_p), ("view_words", C.c_void_p)]


_P = C.c_void_p
_FP = C.POINTER(gift_fif)
class gift_plan_tuning(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int32), ("list_tile", C.c_int32),
                ("narrow_max", C.c_int32), ("gemm", C.c_int32)]


_TP = C.POINTER(gift_plan_tuning)
_VP = C.POINTER(gift_views)
_QP = C.POINTER(gift_queries)
_sig = {
    "gift_version": (C.c_char_p, []),
    "gift_copy_async": (C.c_int32, [_P, _P, C.c_size_t, _P]),
    "gift_last_error": (C.c_char_p, []),
    "gift_quantize_views": (C.c_int32, [_P, C.c_int64, C.c_int32, C.c_int32, _P, _P, _P]),
    "gift_score_exhaustive_workspace": (C.c_size_t, [_VP, _QP]),
    "gift_score_exhaustive": (C.c_int32, [_VP, _QP, _P, _P, C.c_size_t, _P]),
    "gift_query_exhaustive_workspace": (C.c_size_t, [_VP, _QP, C.c_int32, C.c_int32]),
    "gift_query_exhaustive": (C.c_int32, [_VP, _QP, C.c_int32, C.c_int32, _P, _P, _P, _P,
                                          C.c_size_t, _P]),
    "gift_query_exhaustive_static_bytes": (C.c_size_t, [_VP, _QP, C.c_int32, C.c_int32]),
    "gift_query_exhaustive_static": (C.c_int32, [_VP, _QP, C.c_int32, C.c_int32, _P, _P, _P,
                                                 _P]),
    "gift_assign_workspace": (C.c_size_t, [C.c_int64, C.c_int32, C.c_int32, C.c_int32]),
    "gift_assign": (C.c_int32, [_P, C.c_int64, C.c_int32, _P, C.c_int32, C.c_int32, _P, _P, _P,
                                C.c_size_t, _P]),
    "gift_build_codebook_workspace": (C.c_size_t, [C.c_int64, C.c_int32, C.c_int32]),
    "gift_build_codebook": (C.c_int32, [_P, C.c_int64, C.c_int32, C.c_int32, _P, C.c_int32, _P,
                                        _P, C.POINTER(C.c_int32), _P, C.c_size_t, _P]),
    "gift_build_fif_workspace": (C.c_size_t, [_VP, C.c_int32, C.c_int32]),
    "gift_build_fif": (C.c_int32, [_VP, _P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P,
                                   C.c_size_t, _P]),
    "gift_query_fif_workspace": (C.c_size_t, [_VP, _FP, _QP, C.c_int32, C.c_int32]),
    "gift_query_fif": (C.c_int32, [_VP, _FP, _QP, C.c_int32, C.c_int32, _P, _P, _P, _P,
                                   C.c_size_t, _P]),
    "gift_score_fif_workspace": (C.c_size_t, [_VP, _FP, _QP]),
    "gift_score_fif": (C.c_int32, [_VP, _FP, _QP, _P, _P, _P, C.c_size_t, _P]),
    "gift_build_sif_workspace": (C.c_size_t, [C.c_int64]),
    "gift_build_sif": (C.c_int32, [C.c_int64, C.c_int32, _P, _P, _P, _P, _P, _P, _P, C.c_size_t,
                                   _P]),
    "gift_augment_neighbours": (C.c_int32, [C.c_int64, C.c_int32, _P, _P, C.c_int32, _P,
                                            C.c_int32, _P, _P, C.c_int32, _P, _P, C.c_int32, _P,
                                            _P]),
    "gift_fuse_self": (C.c_int32, [C.c_int32, _P, _P, _P, _P, C.c_float, _P, _P]),
    "gift_fuse_activations": (C.c_int32, [C.c_int32, _P, _P, C.c_int32, _P, _P, C.c_int32,
                                          C.c_float, _P, _P, C.c_int32, _P]),
    "gift_rerank_sif": (C.c_int32, [C.c_int64, _P, _P, _P, _P, C.c_int32, C.c_int32, _P, _P, _P,
                                    C.c_int32, _P, _P, _P, _P]),
    "gift_set_score_tuning": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32]),
    "gift_get_score_tuning": (C.c_int32, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "gift_autotune_score": (C.c_int32, [_VP, _QP, _P, C.c_int32, _P, C.c_int32, C.c_int32, _P,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P,
                                        C.c_size_t, _P]),
    "gift_fif_plan_workspace": (C.c_size_t, [_VP, _FP, C.c_int32, C.c_int64, C.c_int32,
                                             C.c_int32, _TP]),
    "gift_fif_plan_create": (C.c_int32, [_VP, _FP, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                         C.c_int32, _P, _P, _P, _P, _P, _TP, _P,
                                         C.c_size_t, _P, C.POINTER(C.c_void_p)]),
    "gift_fif_plan_run": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int64, _P]),
    "gift_fif_plan_serve": (C.c_int32, [C.c_void_p, _P, _P, C.c_int32, C.c_int64, C.c_int64,
                                        _P, _P, _P, _P, _P, C.c_int32, _P, _P, _P, _P, _P,
                                        _P, _P]),
    "gift_fif_plan_run_eager": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int64, _P]),
    "gift_fif_plan_first_pass": (C.c_int32, [C.c_void_p, C.c_int32, _P, _P]),
    "gift_fif_plan_error": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), _P]),
    "gift_fif_plan_phase_us": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), _P]),
    "gift_fif_plan_phase_end_us": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), _P]),
    "gift_fif_plan_destroy": (C.c_int32, [C.c_void_p]),
    "gift_profile_enable": (C.c_int32, [C.c_int32]),
    "gift_profile_reset": (C.c_int32, []),
    "gift_profile_read": (C.c_int32, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "gift_profile_tag_name": (C.c_char_p, [C.c_int32]),
    "gift_probe_mfma": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, _P, _P,
                                    C.POINTER(C.c_int32), _P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    return sorted(_sig)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _check(status):
    if status != OK:
        raise GiftError(status, _lib.gift_last_error().decode())


def copy_async(dst, src, stream=None):
    """Queues dst.copy_(src) on `stream` (device or pinned host tensors of
    the same byte size, contiguous) through gift_copy_async."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n or not (dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("copy_async needs contiguous tensors of the same byte size")
    _check(_lib.gift_copy_async(_ptr(dst), _ptr(src), n, _stream(stream)))


def fif_plan_serve(*args):
    """gift_fif_plan_serve with its 19 arguments already as C-compatible
    values (handles, integer addresses, sizes): a serving loop computes the
    fixed ones once per slot and passes them with the batch sizes."""
    _check(_lib.gift_fif_plan_serve(*args))


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def gift_version() -> str:
    return _lib.gift_version().decode()


class Views:
    """Database views with their storage metadata (keeps tensors alive)."""

    def __init__(self, data, n_views, dtype=F32, scale=None, master=None):
        assert data.is_cuda and data.is_contiguous()
        self.data, self.scale = data, scale
        self.master = master if master is not None else (data if dtype == F32 else None)
        self.dtype, self.n_views = dtype, int(n_views)
        self.dim = int(data.shape[1]) * (2 if dtype == MXFP4 else 1)
        self.n_shapes = int(data.shape[0]) // self.n_views
        self.c = gift_views(data.data_ptr(), dtype, self.n_views, self.n_shapes, self.dim, 0,
                            scale.data_ptr() if scale is not None else None,
                            self.master.data_ptr() if self.master is not None else None)


class Queries:
    """A ragged batch of query view sets (keeps tensors alive)."""

    def __init__(self, views, offsets, max_views=None, offsets_host=None):
        assert views.is_cuda and views.dtype == torch.float32 and views.is_contiguous()
        self.views = views
        if offsets_host is None:
            offsets_host = offsets.cpu() if offsets.is_cuda else offsets
        self.offsets = offsets.to(device=views.device, dtype=torch.int32).contiguous()
        oh = offsets_host.to(torch.int64)
        self.n_queries = int(oh.numel() - 1)
        self.total = int(oh[-1])
        self.max_views = int(max_views if max_views is not None else (oh[1:] - oh[:-1]).max())
        self.c = gift_queries(views.data_ptr(), self.offsets.data_ptr(), self.n_queries,
                              self.max_views, self.total)


def gift_quantize_views(src, dtype, stream=None):
    """Reduced-precision codes of float32 rows: (codes, scale).  BF16 / e4m3:
    per-view float32 scale [n]; MX: uint8 E8M0 [n, dim/32] and codes of
    dim (MXFP8) or dim/2 (MXFP4) bytes per row."""
    n, dim = src.shape
    width = dim // 2 if dtype == MXFP4 else dim
    codes = torch.empty((n, width), dtype=_DT_TORCH[dtype], device=src.device)
    if dtype in (MXFP8, MXFP4):
        scale = torch.empty((n, dim // 32), dtype=torch.uint8, device=src.device)
    else:
        scale = torch.empty(n, dtype=torch.float32, device=src.device)
    _check(_lib.gift_quantize_views(_ptr(src), n, dim, dtype, _ptr(codes), _ptr(scale),
                                    _stream(stream)))
    return codes, scale


def gift_score_exhaustive(db: Views, q: Queries, stream=None):
    """First-pass Eq. 3 scores [B, N] float32 in the database's dtype."""
    ws = _workspace(_lib.gift_score_exhaustive_workspace(C.byref(db.c), C.byref(q.c)),
                    db.data.device)
    out = torch.empty((q.n_queries, db.n_shapes), dtype=torch.float32, device=db.data.device)
    _check(_lib.gift_score_exhaustive(C.byref(db.c), C.byref(q.c), _ptr(out), _ptr(ws),
                                      ws.numel(), _stream(stream)))
    return out


def gift_query_exhaustive(db: Views, q: Queries, top_k, rescore_r, stream=None, ws=None):
    """Exact top-k of Eq. 3: (ids int32 [B,k], scores f32 [B,k], flags int32 [B])."""
    dev = db.data.device
    need = _lib.gift_query_exhaustive_workspace(C.byref(db.c), C.byref(q.c), top_k, rescore_r)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    ids = torch.empty((q.n_queries, top_k), dtype=torch.int32, device=dev)
    scores = torch.empty((q.n_queries, top_k), dtype=torch.float32, device=dev)
    flags = torch.empty(q.n_queries, dtype=torch.int32, device=dev)
    _check(_lib.gift_query_exhaustive(C.byref(db.c), C.byref(q.c), top_k, rescore_r,
                                      _ptr(ids), _ptr(scores), _ptr(flags), _ptr(ws),
                                      ws.numel(), _stream(stream)))
    return ids, scores, flags


# size of the static device scratch behind gift_query_exhaustive_static
STATIC_SCRATCH_BYTES = 64 << 20


def gift_query_exhaustive_static(db: Views, q: Queries, top_k, rescore_r, stream=None,
                                 out=None):
    """gift_query_exhaustive on the library's static device scratch (no
    workspace, no device allocation inside the call).  `out` = (ids, scores,
    flags) preallocated outputs, or None to allocate them here."""
    dev = db.data.device
    if out is None:
        out = (torch.empty((q.n_queries, top_k), dtype=torch.int32, device=dev),
               torch.empty((q.n_queries, top_k), dtype=torch.float32, device=dev),
               torch.empty(q.n_queries, dtype=torch.int32, device=dev))
    ids, scores, flags = out
    _check(_lib.gift_query_exhaustive_static(C.byref(db.c), C.byref(q.c), top_k, rescore_r,
                                             _ptr(ids), _ptr(scores), _ptr(flags),
                                             _stream(stream)))
    return ids, scores, flags


def query_exhaustive_static_bytes(db: Views, q: Queries, top_k, rescore_r) -> int:
    return int(_lib.gift_query_exhaustive_static_bytes(C.byref(db.c), C.byref(q.c), top_k,
                                                       rescore_r))


def query_exhaustive_workspace(db: Views, q: Queries, top_k, rescore_r) -> int:
    return int(_lib.gift_query_exhaustive_workspace(C.byref(db.c), C.byref(q.c), top_k,
                                                    rescore_r))


PROFILE_TAGS = {"quantize": 0, "score_tiles": 1, "reduce_queries": 2, "select_top": 3,
                "rescore": 4, "final_rank": 5, "assign": 6, "group_queries": 7, "fif_scan": 8,
                "rerank_sif": 9}


def gift_profile_enable(capacity: int):
    _check(_lib.gift_profile_enable(int(capacity)))


def gift_profile_reset():
    _check(_lib.gift_profile_reset())


def gift_probe_mfma(dtype: int, blocks: int, iters: int, stream=None):
    """Launches the MFMA rate probe; returns (sink, clocks, wall_khz): device
    tensors (clocks: [blocks, 2] int64 of clock64 and wall_clock64 deltas)
    and the wall clock's rate in kHz."""
    dev = torch.device("cuda", torch.cuda.current_device())
    sink = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    clocks = torch.empty((blocks, 2), dtype=torch.int64, device=dev)
    khz = C.c_int32(0)
    _check(_lib.gift_probe_mfma(dtype, blocks, iters, _ptr(sink), _ptr(clocks), C.byref(khz),
                                _stream(stream)))
    return sink, clocks, khz.value


def gift_profile_read(tag: str):
    """(total ms, launch count) of the recorded launches of one kernel."""
    tot, cnt = C.c_double(), C.c_int32()
    _check(_lib.gift_profile_read(PROFILE_TAGS[tag], C.byref(tot), C.byref(cnt)))
    return tot.value, cnt.value


# ---------------------------------------------------------------- F-IF
def gift_assign(x, codebook, ma=1, stream=None):
    """Words [n, ma] int32 of the rows of x (Sec. 2.3 quantizer) and the
    device count of uncertified rows."""
    n, dim = x.shape
    K = int(codebook.shape[0])
    ws = _workspace(_lib.gift_assign_workspace(n, dim, K, ma), x.device)
    words = torch.empty((n, ma), dtype=torch.int32, device=x.device)
    unc = torch.zeros(1, dtype=torch.int32, device=x.device)
    _check(_lib.gift_assign(_ptr(x), n, dim, _ptr(codebook), K, ma, _ptr(words), _ptr(unc),
                            _ptr(ws), ws.numel(), _stream(stream)))
    return words, unc


def gift_build_codebook(train, K, init_idx, max_iter=25, stream=None):
    """k-means vocabulary: (codebook [K, d] f32, assign [n] i32, iterations)."""
    n, dim = train.shape
    init = torch.as_tensor(init_idx, dtype=torch.int64).cpu().contiguous()
    ws = _workspace(_lib.gift_build_codebook_workspace(n, dim, K), train.device)
    cb = torch.empty((K, dim), dtype=torch.float32, device=train.device)
    a = torch.empty(n, dtype=torch.int32, device=train.device)
    it = C.c_int32(0)
    _check(_lib.gift_build_codebook(_ptr(train), n, dim, K, C.c_void_p(init.data_ptr()),
                                    max_iter, _ptr(cb), _ptr(a), C.byref(it), _ptr(ws),
                                    ws.numel(), _stream(stream)))
    return cb, a, it.value


class Fif:
    """A first inverted file and its codebook (keeps tensors alive)."""

    def __init__(self, codebook, ma, offsets, entry_shape, entry_view, view_words):
        self.codebook, self.ma = codebook, int(ma)
        self.K = int(codebook.shape[0])
        self.offsets, self.entry_shape, self.entry_view = offsets, entry_shape, entry_view
        self.view_words = view_words
        self.c = gift_fif(codebook.data_ptr(), self.K, self.ma, int(entry_shape.numel()),
                          offsets.data_ptr(), entry_shape.data_ptr(), entry_view.data_ptr(),
                          view_words.data_ptr())


def gift_build_fif(db: Views, codebook, ma=1, stream=None):
    K = int(codebook.shape[0])
    dev = db.data.device
    nv = db.n_shapes * db.n_views
    ws = _workspace(_lib.gift_build_fif_workspace(C.byref(db.c), K, ma), dev)
    off = torch.empty(K + 1, dtype=torch.int64, device=dev)
    es = torch.empty(nv * ma, dtype=torch.int32, device=dev)
    ev = torch.empty(nv * ma, dtype=torch.int32, device=dev)
    vw = torch.empty((nv, ma), dtype=torch.int32, device=dev)
    _check(_lib.gift_build_fif(C.byref(db.c), _ptr(codebook), K, ma, _ptr(off), _ptr(es),
                               _ptr(ev), _ptr(vw), _ptr(ws), ws.numel(), _stream(stream)))
    return Fif(codebook, ma, off, es, ev, vw)


def gift_query_fif(db: Views, fif: Fif, q: Queries, top_k, rescore_r, stream=None, ws=None):
    """Exact top-k of Eq. 4: (ids, scores, flags)."""
    dev = db.data.device
    need = _lib.gift_query_fif_workspace(C.byref(db.c), C.byref(fif.c), C.byref(q.c), top_k,
                                         rescore_r)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    ids = torch.empty((q.n_queries, top_k), dtype=torch.int32, device=dev)
    scores = torch.empty((q.n_queries, top_k), dtype=torch.float32, device=dev)
    flags = torch.empty(q.n_queries, dtype=torch.int32, device=dev)
    _check(_lib.gift_query_fif(C.byref(db.c), C.byref(fif.c), C.byref(q.c), top_k, rescore_r,
                               _ptr(ids), _ptr(scores), _ptr(flags), _ptr(ws), ws.numel(),
                               _stream(stream)))
    return ids, scores, flags


def query_fif_workspace(db: Views, fif: Fif, q: Queries, top_k, rescore_r) -> int:
    return int(_lib.gift_query_fif_workspace(C.byref(db.c), C.byref(fif.c), C.byref(q.c),
                                             top_k, rescore_r))


def gift_score_fif(db: Views, fif: Fif, q: Queries, stream=None):
    """First-pass Eq. 4 scores [B, N] and the query words [total_views]."""
    dev = db.data.device
    ws = _workspace(_lib.gift_score_fif_workspace(C.byref(db.c), C.byref(fif.c), C.byref(q.c)),
                    dev)
    out = torch.empty((q.n_queries, db.n_shapes), dtype=torch.float32, device=dev)
    qw = torch.empty(q.total, dtype=torch.int32, device=dev)
    _check(_lib.gift_score_fif(C.byref(db.c), C.byref(fif.c), C.byref(q.c), _ptr(out), _ptr(qw),
                               _ptr(ws), ws.numel(), _stream(stream)))
    return out, qw


# ---------------------------------------------------------------- S-IF
class Sif:
    """The second inverted file (keeps tensors alive)."""

    def __init__(self, n_shapes, l1, post_off, post_id, post_val):
        self.n_shapes = int(n_shapes)
        self.l1, self.post_off, self.post_id, self.post_val = l1, post_off, post_id, post_val

    def nnz(self):
        return int(self.post_off[-1].item())


def gift_build_sif(nbr_ids, nbr_scores, stream=None):
    """S-IF from neighbour lists [N, k1] (int32 ids, float32 scores)."""
    N, k1 = nbr_ids.shape
    dev = nbr_ids.device
    ws = _workspace(_lib.gift_build_sif_workspace(N), dev)
    l1 = torch.empty((N, 2), dtype=torch.float32, device=dev)
    off = torch.empty(N + 1, dtype=torch.int64, device=dev)
    pid = torch.empty(N * k1, dtype=torch.int32, device=dev)
    pval = torch.empty(N * k1, dtype=torch.float32, device=dev)
    _check(_lib.gift_build_sif(N, k1, _ptr(nbr_ids), _ptr(nbr_scores), _ptr(l1), _ptr(off),
                               _ptr(pid), _ptr(pval), _ptr(ws), ws.numel(), _stream(stream)))
    return Sif(N, l1, off, pid, pval)


def gift_rerank_sif(sif: Sif, q_ids, q_scores, q_self, top_k, stream=None):
    """Top-k by Eq. 8 for each query's activation: (ids, scores, flags)."""
    B, k1 = q_ids.shape
    dev = q_ids.device
    ids = torch.empty((B, top_k), dtype=torch.int32, device=dev)
    scores = torch.empty((B, top_k), dtype=torch.float32, device=dev)
    flags = torch.empty(B, dtype=torch.int32, device=dev)
    _check(_lib.gift_rerank_sif(sif.n_shapes, _ptr(sif.l1), _ptr(sif.post_off), _ptr(sif.post_id),
                                _ptr(sif.post_val), B, k1, _ptr(q_ids), _ptr(q_scores),
                                _ptr(q_self), top_k, _ptr(ids), _ptr(scores), _ptr(flags),
                                _stream(stream)))
    return ids, scores, flags


# ---------------------------------------------------------------- tuning
def gift_set_score_tuning(dtype, tile, group):
    _check(_lib.gift_set_score_tuning(dtype, tile, group))


def gift_get_score_tuning(dtype):
    t, g = C.c_int32(), C.c_int32()
    _check(_lib.gift_get_score_tuning(dtype, C.byref(t), C.byref(g)))
    return t.value, g.value


def gift_autotune_score(db: Views, q: Queries, tiles, groups, reps=2, stream=None):
    """Times every (tile, group) pair on this workload and selects the best.
    Returns (best_tile, best_group, ms [len(tiles), len(groups)])."""
    import numpy as np
    ti = (C.c_int32 * len(tiles))(*tiles)
    gr = (C.c_int32 * len(groups))(*groups)
    ms = (C.c_float * (len(tiles) * len(groups)))()
    bt, bg = C.c_int32(), C.c_int32()
    ws = _workspace(_lib.gift_score_exhaustive_workspace(C.byref(db.c), C.byref(q.c)),
                    db.data.device)
    _check(_lib.gift_autotune_score(C.byref(db.c), C.byref(q.c), ti, len(tiles), gr, len(groups),
                                    reps, ms, C.byref(bt), C.byref(bg), _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return bt.value, bg.value, np.array(ms[:], dtype=np.float32).reshape(len(tiles), len(groups))


# ---------------------------------------------------------------- plans
def plan_tuning(blocks_per_cu=2, list_tile=128, narrow_max=32, gemm=0):
    """gemm: 0 placed by capacity, 1 inside the persistent kernel, 2 a
    separate GEMM kernel."""
    return gift_plan_tuning(int(blocks_per_cu), int(list_tile), int(narrow_max), int(gemm))


def fif_plan_workspace(db: Views, fif: Fif, max_queries, max_views, top_k, rescore_r,
                       tuning=None) -> int:
    t = tuning if tuning is not None else plan_tuning()
    return int(_lib.gift_fif_plan_workspace(C.byref(db.c), C.byref(fif.c), max_queries,
                                            max_views, top_k, rescore_r, C.byref(t)))


class FifPlan:
    """A captured F-IF batch plan with its own input/output buffers.

    Fill ``views[:n_views]`` and ``offsets[:n_queries + 1]`` (device) and call
    ``run(n_queries, n_views)``; results land in ``ids``, ``scores``,
    ``flags``.  The plan captures on (and by default runs on) its own
    non-default stream."""

    def __init__(self, db: Views, fif: Fif, max_queries, max_views, max_views_per_query, top_k,
                 rescore_r, blocks_per_cu=2, stream=None, ws=None, views=None, list_tile=128,
                 narrow_max=32, gemm=0):
        """ws (uint8) and views (float32 [max_views, dim]) may be given as
        caller-owned device tensors (e.g. carved from a memory pool); they
        must outlive the plan."""
        dev = db.data.device
        self.db, self.fif = db, fif
        self.max_queries, self.max_views, self.top_k = max_queries, max_views, top_k
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        if views is not None:
            assert views.shape == (max_views, db.dim) and views.dtype == torch.float32
            self.views = views
        else:
            self.views = torch.zeros((max_views, db.dim), dtype=torch.float32, device=dev)
        self.offsets = torch.zeros(max_queries + 1, dtype=torch.int32, device=dev)
        self.ids = torch.zeros((max_queries, top_k), dtype=torch.int32, device=dev)
        self.scores = torch.zeros((max_queries, top_k), dtype=torch.float32, device=dev)
        self.flags = torch.zeros(max_queries, dtype=torch.int32, device=dev)
        self.tuning = plan_tuning(blocks_per_cu, list_tile, narrow_max, gemm)
        need = fif_plan_workspace(db, fif, max_queries, max_views, top_k, rescore_r, self.tuning)
        if ws is not None:
            assert ws.dtype == torch.uint8 and ws.numel() >= need
            self.ws = ws
        else:
            self.ws = _workspace(need, dev)
        torch.cuda.synchronize(dev)
        self.handle = C.c_void_p()
        _check(_lib.gift_fif_plan_create(C.byref(db.c), C.byref(fif.c), max_queries, max_views,
                                         max_views_per_query, top_k, rescore_r,
                                         _ptr(self.views), _ptr(self.offsets), _ptr(self.ids),
                                         _ptr(self.scores), _ptr(self.flags),
                                         C.byref(self.tuning),
                                         _ptr(self.ws), self.ws.numel(), _stream(self.stream),
                                         C.byref(self.handle)))

    def run(self, n_queries, n_views, stream=None, eager=False):
        f = _lib.gift_fif_plan_run_eager if eager else _lib.gift_fif_plan_run
        _check(f(self.handle, n_queries, n_views, _stream(stream or self.stream)))

    def first_pass(self, n_queries, stream=None):
        """First-pass Eq. 4 scores [n_queries, n_shapes] of the last run."""
        out = torch.empty((n_queries, self.db.n_shapes), dtype=torch.float32,
                          device=self.db.data.device)
        _check(_lib.gift_fif_plan_first_pass(self.handle, n_queries, _ptr(out),
                                             _stream(stream or self.stream)))
        return out

    def phase_us(self, stream=None):
        """Block-microseconds per phase of the last run, waits for inputs
        excluded (split and quantize, codeword dots, clear, word selection,
        word offsets, grouping, active-tile listing, list scan, per-query
        mean; the clear runs inside the codeword-dot items and reads 0)."""
        out = (C.c_double * 9)()
        _check(_lib.gift_fif_plan_phase_us(self.handle, out, _stream(stream or self.stream)))
        return list(out)

    def phase_end_us(self, stream=None):
        """Microseconds from the start of the last run to the end of each
        phase's last item, in the order of phase_us."""
        out = (C.c_double * 9)()
        _check(_lib.gift_fif_plan_phase_end_us(self.handle, out, _stream(stream or self.stream)))
        return list(out)

    def error(self, stream=None):
        e = C.c_int32()
        _check(_lib.gift_fif_plan_error(self.handle, C.byref(e), _stream(stream or self.stream)))
        return e.value

    def close(self):
        if self.handle:
            _lib.gift_fif_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gift_augment_neighbours(nbr_ids, nbr_scores, members, own_ids=None, own_scores=None,
                            k_out=None, stream=None):
    """Eq. 10 rows: (ids [n, k_out], scores [n, k_out], n_members [n])."""
    N, k1 = nbr_ids.shape
    n_rows, k2 = members.shape
    k_own = int(own_ids.shape[1]) if own_ids is not None else 0
    k_out = k_out or (k2 * k1 + k_own)
    dev = nbr_ids.device
    oi = torch.empty((n_rows, k_out), dtype=torch.int32, device=dev)
    os_ = torch.empty((n_rows, k_out), dtype=torch.float32, device=dev)
    nm = torch.empty(n_rows, dtype=torch.int32, device=dev)
    _check(_lib.gift_augment_neighbours(N, k1, _ptr(nbr_ids), _ptr(nbr_scores), n_rows,
                                        _ptr(members), k2, _ptr(own_ids), _ptr(own_scores), k_own,
                                        _ptr(oi), _ptr(os_), k_out, _ptr(nm), _stream(stream)))
    return oi, os_, nm


def gift_fuse_self(self1, n1, self2, n2, alpha=0.5, stream=None):
    """Fused self membership [n] of outside queries (Eq. 11 then Eq. 9)."""
    n = int(self1.shape[0])
    out = torch.empty(n, dtype=torch.float32, device=self1.device)
    _check(_lib.gift_fuse_self(n, _ptr(self1), _ptr(n1), _ptr(self2), _ptr(n2), float(alpha),
                               _ptr(out), _stream(stream)))
    return out


def gift_fuse_activations(ids1, sc1, ids2, sc2, alpha=0.5, k_out=None, stream=None):
    """Eq. 9 rows: (ids [n, k_out], scores [n, k_out])."""
    n, k_a = ids1.shape
    k_b = int(ids2.shape[1])
    k_out = k_out or (k_a + k_b)
    oi = torch.empty((n, k_out), dtype=torch.int32, device=ids1.device)
    os_ = torch.empty((n, k_out), dtype=torch.float32, device=ids1.device)
    _check(_lib.gift_fuse_activations(n, _ptr(ids1), _ptr(sc1), k_a, _ptr(ids2), _ptr(sc2), k_b,
                                      float(alpha), _ptr(oi), _ptr(os_), k_out, _stream(stream)))
    return oi, os_
