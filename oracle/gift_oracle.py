"""Plain CPU oracle of GIFT's search stage (arXiv 1604.01879).

TEST INFRASTRUCTURE ONLY.  Nothing in the product imports this module; only
the tests, the smoke check and the CPU-baseline leg of the benchmark call it.
It shares no code, header, table or helper with the GPU path.

Everything is numpy.  Floating point is float64 over the float32 inputs
unless a function says otherwise: products of two float32 values are exact in
float64, so the only rounding left is the float64 summation (relative error
around 1e-13 at d = 4096).  Library matmuls are used as the dot-product step;
there is no other blocking, fusion or reordering.

Readings of points the paper leaves open are marked READING where they are
applied, each with the choice it makes.
"""
from __future__ import annotations

import numpy as np

f64 = np.float64
f32 = np.float32

__all__ = [
    "similarity", "exhaustive_scores", "exhaustive_scores_literal",
    "rank_topk", "quantizer_dist", "assign", "kmeans", "build_fif",
    "fif_scores", "fif_scores_literal", "build_sif", "rerank_sif",
    "rerank_sif_dense", "jaccard_dense", "quantize_views", "dequantize",
    "lowprec_exhaustive_scores", "recall_at_k", "self_score",
    "neighbour_augment", "fuse_activations", "co_augment", "quantize_views_mx",
    "dequantize_mx",
]


# --------------------------------------------------------------------------
# Sec. 2.3, Eq. 3: multi-view matching
# --------------------------------------------------------------------------

def similarity(q: np.ndarray, p: np.ndarray, dtype=f64) -> np.ndarray:
    """s(q_i, p_j) for all pairs: cosine similarity (Sec. 2.3, after Eq. 3).

    Features are L2-normalised when they are extracted (Sec. 2.2), so the
    cosine is the dot product of the stored vectors.  READING: no
    renormalisation happens here; both sides read the same float32 bits.
    """
    return np.asarray(q, dtype=dtype) @ np.asarray(p, dtype=dtype).T


def _query_slices(qoff):
    qoff = np.asarray(qoff)
    return [(int(qoff[b]), int(qoff[b + 1])) for b in range(len(qoff) - 1)]


def exhaustive_scores(qviews, qoff, db, n_views, dtype=f64, shape_chunk=256):
    """Eq. 3 for every (query, database shape): S[b, p].

    S(x_q, x_p) = (1/m) * sum_i max_j s(q_i, p_j), where m is the number of
    views of the query (READING: the paper's 1/N_v with N_v = |V(x_q)|).
    The sum over query views runs in ascending i.
    db is [N*Nv, d] shape-major.  Returns float64 (or ``dtype``) [B, N].
    """
    db = np.asarray(db)
    n_shapes = db.shape[0] // n_views
    sl = _query_slices(qoff)
    out = np.zeros((len(sl), n_shapes), dtype=dtype)
    for s0 in range(0, n_shapes, shape_chunk):
        s1 = min(n_shapes, s0 + shape_chunk)
        P = np.asarray(db[s0 * n_views:s1 * n_views], dtype=dtype)
        for b, (lo, hi) in enumerate(sl):
            m = hi - lo
            if m == 0:
                continue
            sim = similarity(qviews[lo:hi], P, dtype)          # [m, ns*Nv]
            best = sim.reshape(m, s1 - s0, n_views).max(axis=2)  # max over j
            acc = np.zeros(s1 - s0, dtype=dtype)
            for i in range(m):                                 # ascending i
                acc = acc + best[i]
            out[b, s0:s1] = acc / dtype(m)
    return out


def exhaustive_scores_literal(qviews, qoff, db, n_views):
    """Eq. 3 as a pure-Python triple loop (tiny inputs only)."""
    db = np.asarray(db, dtype=f64)
    n_shapes = db.shape[0] // n_views
    res = []
    for lo, hi in _query_slices(qoff):
        row = []
        for p in range(n_shapes):
            tot = 0.0
            for i in range(lo, hi):
                best = -np.inf
                for j in range(n_views):
                    v = float(np.dot(np.asarray(qviews[i], f64), db[p * n_views + j]))
                    best = max(best, v)
                tot += best
            row.append(tot / (hi - lo))
        res.append(row)
    return np.array(res, dtype=f64)


def self_score(qviews, qoff, dtype=f64):
    """S(x_q, x_q) by Eq. 3 with the query as its own database shape."""
    out = []
    for lo, hi in _query_slices(qoff):
        sim = similarity(qviews[lo:hi], qviews[lo:hi], dtype)
        best = sim.max(axis=1)
        acc = dtype(0)
        for i in range(hi - lo):
            acc = acc + best[i]
        out.append(acc / dtype(hi - lo))
    return np.array(out, dtype=dtype)


# --------------------------------------------------------------------------
# Ranking list (Sec. 1 and the top-k neighbour sets of Sec. 2.4)
# --------------------------------------------------------------------------

def rank_topk(scores: np.ndarray, k: int):
    """Top-k of each row by (score descending, shape id ascending).

    READING: ties go to the lower id; every shape takes part, so zero scores
    pad the list in id order.  Returns (ids int32 [B, k], scores [B, k]).
    """
    scores = np.atleast_2d(scores)
    B, N = scores.shape
    k = min(k, N)
    ids = np.empty((B, k), dtype=np.int32)
    vals = np.empty((B, k), dtype=scores.dtype)
    idx = np.arange(N)
    for b in range(B):
        order = np.lexsort((idx, -scores[b]))[:k]
        ids[b] = order
        vals[b] = scores[b, order]
    return ids, vals


# --------------------------------------------------------------------------
# Sec. 2.3: quantizer c(x) = argmin_k ||x - b_k||^2, Multiple Assignment
# --------------------------------------------------------------------------

def quantizer_dist(x, codebook, direct=False):
    """Squared Euclidean distance from each row of x to each codeword (f64).

    The expansion ||b||^2 - 2 x.b + ||x||^2 is used by default; ``direct``
    forms ||x - b||^2 literally (tiny inputs only).
    """
    X = np.asarray(x, dtype=f64)
    Bk = np.asarray(codebook, dtype=f64)
    if direct:
        diff = X[:, None, :] - Bk[None, :, :]
        return np.einsum("nkd,nkd->nk", diff, diff)
    xx = np.einsum("nd,nd->n", X, X)
    bb = np.einsum("kd,kd->k", Bk, Bk)
    return (bb[None, :] - 2.0 * (X @ Bk.T)) + xx[:, None]


def assign(x, codebook, ma=1, chunk=8192):
    """c(x) (ma=1) or the ma nearest codewords (Multiple Assignment).

    The nearest codewords are ordered by (distance, codeword index), so equal
    distances go to the lower index (READING).  Returns int32 [n, ma].
    """
    X = np.asarray(x)
    n = X.shape[0]
    K = np.asarray(codebook).shape[0]
    if ma > K:
        raise ValueError("ma > K")
    out = np.empty((n, ma), dtype=np.int32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        d = quantizer_dist(X[lo:hi], codebook)
        out[lo:hi] = np.argsort(d, axis=1, kind="stable")[:, :ma]
    return out


def kmeans(train, init_idx, max_iter=25):
    """Lloyd's k-means for the vocabulary B = {b_1..b_K} (Sec. 2.3).

    The paper names k-means only (it is the costliest offline step after CNN
    training, Sec. 3.4).  READING: Lloyd iterations from the K training rows
    ``init_idx``; assignment by ``assign`` (ma=1); each centroid is the mean
    of its members, summed in float64 in ascending member order and divided
    in float64, then rounded once to float32; an empty cluster keeps its
    previous centroid; stop when no assignment changes or after
    ``max_iter`` updates.  Returns (codebook f32 [K, d], assign int32 [n],
    iterations run).
    """
    X = np.asarray(train, dtype=f32)
    B = X[np.asarray(init_idx)].copy()
    a = assign(X, B, 1)[:, 0]
    it = 0
    for it in range(1, max_iter + 1):
        newB = B.copy()
        for k in range(B.shape[0]):
            members = np.flatnonzero(a == k)          # ascending row order
            if members.size == 0:
                continue
            s = np.zeros(X.shape[1], dtype=f64)
            for r in members:
                s = s + X[r].astype(f64)
            newB[k] = (s / f64(members.size)).astype(f32)
        B = newB
        a_new = assign(X, B, 1)[:, 0]
        changed = int(np.count_nonzero(a_new != a))
        a = a_new
        if changed == 0:
            break
    return B, a.astype(np.int32), it


# --------------------------------------------------------------------------
# Sec. 2.3, Eq. 4 and Fig. 2: the first inverted file (F-IF)
# --------------------------------------------------------------------------

def build_fif(db_words: np.ndarray, K: int, n_views: int):
    """The first inverted file from per-view word lists (Sec. 2.3, Fig. 2).

    db_words[v] holds the MA words of database view v = p*Nv + j.  Each view
    is stored once in every one of its words' entries, with its shape id
    (READING: MA applies on the database side).  Entries of a word are in
    ascending (shape, view) order.  Returns (offsets int64 [K+1],
    entry_shape int32, entry_view int32).
    """
    W = np.asarray(db_words)
    ma = W.shape[1]
    flat = W.reshape(-1)
    order = np.argsort(flat, kind="stable")
    counts = np.bincount(flat, minlength=K)
    offsets = np.zeros(K + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    views = (order // ma).astype(np.int64)
    return offsets, (views // n_views).astype(np.int32), (views % n_views).astype(np.int32)


def fif_scores(qviews, qoff, db, n_views, codebook, offsets, entry_shape,
               entry_view, dtype=f64, qwords=None):
    """Eq. 4 through list scans: S_F[b, p].

    Each query view q_i is hard-assigned to its nearest word w_i = c(q_i).
    M_i(p) = max of s(q_i, p_j) over the entries (p, j) of list w_i, or 0 if
    shape p has no view in that list (READING of the Kronecker delta).
    S_F = (1/m) sum_i M_i(p), summed in ascending i.  ``qwords`` may give the
    query words (e.g. decided on float32 views while the dot products use
    dequantised low-precision values).
    """
    db = np.asarray(db)
    n_shapes = db.shape[0] // n_views
    sl = _query_slices(qoff)
    out = np.zeros((len(sl), n_shapes), dtype=dtype)
    for b, (lo, hi) in enumerate(sl):
        m = hi - lo
        if m == 0:
            continue
        if qwords is None:
            words = assign(qviews[lo:hi], codebook, 1)[:, 0]
        else:
            words = np.asarray(qwords[lo:hi])
        acc = np.zeros(n_shapes, dtype=dtype)
        for i in range(m):
            w = words[i]
            e0, e1 = int(offsets[w]), int(offsets[w + 1])
            M = np.zeros(n_shapes, dtype=dtype)
            if e1 > e0:
                shp = entry_shape[e0:e1]
                rows = shp.astype(np.int64) * n_views + entry_view[e0:e1]
                s = similarity(qviews[lo + i:lo + i + 1], db[rows], dtype)[0]
                best = np.full(n_shapes, -np.inf, dtype=dtype)
                np.maximum.at(best, shp, s)
                hit = np.isfinite(best)
                M[hit] = best[hit]
            acc = acc + M
        out[b] = acc / dtype(m)
    return out


def fif_scores_literal(qviews, qoff, db, n_views, codebook, db_words):
    """Eq. 4 as written: max_j s(q_i,p_j) * delta(c(q_i) in C_MA(p_j)).

    Double loop over all view pairs (tiny inputs only).
    """
    db = np.asarray(db, dtype=f64)
    n_shapes = db.shape[0] // n_views
    res = []
    for lo, hi in _query_slices(qoff):
        wq = assign(qviews[lo:hi], codebook, 1)[:, 0]
        row = []
        for p in range(n_shapes):
            tot = 0.0
            for i in range(hi - lo):
                best = -np.inf
                for j in range(n_views):
                    v = p * n_views + j
                    delta = 1.0 if wq[i] in set(int(w) for w in db_words[v]) else 0.0
                    best = max(best, float(np.dot(np.asarray(qviews[lo + i], f64), db[v])) * delta)
                tot += best
            row.append(tot / (hi - lo))
        res.append(row)
    return np.array(res, dtype=f64)


# --------------------------------------------------------------------------
# Sec. 2.4: the second inverted file (S-IF), Eq. 7, 8, 12-14, Fig. 3
# --------------------------------------------------------------------------

def build_sif(nbr_ids: np.ndarray, nbr_scores: np.ndarray, n_shapes: int):
    """The second inverted file from each database shape's top-k1 list.

    F_p[i] = S(x_p, x_i) if x_i is among p's k1 neighbours, else 0 (Eq. 7).
    Entry i stores ||F_i||_1 (the sigma-count of shape i's fuzzy neighbour
    set, pre-computed offline, Eq. 14) and the postings (p, F_p[i]) of the
    shapes whose membership at i is non-zero (READING of "non-negative"),
    in ascending p.  Ids < 0 are padding.
    Returns (l1 f64 [N], post_off int64 [N+1], post_id int32, post_val f64).
    """
    ids = np.asarray(nbr_ids)
    vals = np.asarray(nbr_scores, dtype=f64)
    N = n_shapes
    l1 = np.zeros(N, dtype=f64)
    cols = [[] for _ in range(N)]
    for p in range(ids.shape[0]):
        for r in range(ids.shape[1]):
            i = int(ids[p, r])
            if i < 0:
                continue
            l1[p] += vals[p, r]
            if vals[p, r] > 0:
                cols[i].append((p, vals[p, r]))
    post_off = np.zeros(N + 1, dtype=np.int64)
    pid, pval = [], []
    for i in range(N):
        cols[i].sort(key=lambda t: t[0])
        pid.extend(t[0] for t in cols[i])
        pval.extend(t[1] for t in cols[i])
        post_off[i + 1] = len(pid)
    return l1, post_off, np.array(pid, dtype=np.int32), np.array(pval, dtype=f64)


def rerank_sif(l1, post_off, post_id, post_val, q_ids, q_scores, q_self, top_k):
    """Eq. 8 evaluated through the inverted file (Eq. 13 and 14).

    F_q has the memberships q_scores at coordinates q_ids (ids < 0 skipped),
    plus a membership q_self for the query itself, which is no database
    coordinate and so only enters ||F_q||_1 (READING for queries outside the
    database; pass 0 for a database shape whose own id is in q_ids).
    num[p] = sum over shared non-zero coordinates of min(F_q[i], F_p[i])
    (Eq. 13); S' = num / (||F_q||_1 + ||F_p||_1 - num) (Eq. 14); shapes that
    share nothing score 0.  Returns the top_k by (S' desc, id asc) and the
    dense S' vector.
    """
    N = len(l1)
    num = np.zeros(N, dtype=f64)
    A = float(q_self)
    for i, v in zip(np.asarray(q_ids), np.asarray(q_scores, dtype=f64)):
        if i < 0:
            continue
        A += v
    for i, v in zip(np.asarray(q_ids), np.asarray(q_scores, dtype=f64)):
        if i < 0:
            continue
        for e in range(int(post_off[i]), int(post_off[i + 1])):
            num[post_id[e]] += min(v, post_val[e])
    S = np.zeros(N, dtype=f64)
    nz = num > 0
    S[nz] = num[nz] / (A + l1[nz] - num[nz])
    ids, vals = rank_topk(S[None, :], top_k)
    return ids[0], vals[0], S


def jaccard_dense(Fq: np.ndarray, Fp: np.ndarray) -> float:
    """Eq. 8 on dense membership vectors: sum min / sum max."""
    den = np.maximum(Fq, Fp).sum()
    return float(np.minimum(Fq, Fp).sum() / den) if den > 0 else 0.0


def rerank_sif_dense(nbr_ids, nbr_scores, q_ids, q_scores, q_self, n_shapes):
    """Eq. 8 over explicit length-(N+1) vectors (the last slot is the query
    itself).  Used to check the inverted evaluation."""
    N = n_shapes
    F = np.zeros((nbr_ids.shape[0], N + 1), dtype=f64)
    for p in range(nbr_ids.shape[0]):
        for r in range(nbr_ids.shape[1]):
            if nbr_ids[p, r] >= 0:
                F[p, nbr_ids[p, r]] = nbr_scores[p, r]
    Fq = np.zeros(N + 1, dtype=f64)
    for i, v in zip(q_ids, q_scores):
        if i >= 0:
            Fq[i] = v
    Fq[N] = q_self
    return np.array([jaccard_dense(Fq, F[p]) for p in range(N)], dtype=f64)


def neighbour_augment(F: np.ndarray, nbr_ids: np.ndarray, k2: int) -> np.ndarray:
    """Eq. 10 on dense rows: F_q := mean of F_i over the top-k2 neighbours.

    READING: a Jacobi update (the right side uses the un-augmented rows) and
    the neighbour list includes the shape itself at rank 1, so k2 = 1 leaves
    F unchanged.
    """
    out = np.zeros_like(F)
    for q in range(F.shape[0]):
        nb = [int(i) for i in nbr_ids[q, :k2] if i >= 0]
        for i in nb:
            out[q] += F[i]
        out[q] /= len(nb)
    return out


def co_augment(F1: np.ndarray, F2: np.ndarray, nbr1: np.ndarray, nbr2: np.ndarray, k2: int):
    """Eq. 11: each measure's rows averaged over the other measure's top-k2
    neighbours (Jacobi, un-augmented right-hand sides)."""
    return neighbour_augment(F1, nbr2, k2), neighbour_augment(F2, nbr1, k2)


def fuse_activations(F1: np.ndarray, F2: np.ndarray, alpha: float) -> np.ndarray:
    """Eq. 9: element-wise generalised mean with exponent alpha of two
    activations, ((F1^a + F2^a) / 2)^(1/a), with 0^a = 0 for a > 0."""
    a = float(alpha)
    return ((np.power(F1, a) + np.power(F2, a)) / 2.0) ** (1.0 / a)


# --------------------------------------------------------------------------
# Reduced-precision storage (not in the paper): per-view scaled BF16 / FP8
# --------------------------------------------------------------------------

_FMAX = {"bf16": 1.0, "fp8": 448.0}


def _round_bf16(y: np.ndarray) -> np.ndarray:
    """Round float32 to the nearest bfloat16 (ties to even), as float32."""
    u = np.asarray(y, dtype=f32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(f32)


def _e4m3_grid() -> np.ndarray:
    """All finite non-negative OCP E4M3FN values (bias 7, max 448)."""
    vals = set()
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue                      # NaN encoding
            if e == 0:
                vals.add(m / 8.0 * 2.0 ** -6)  # subnormals
            else:
                vals.add((1 + m / 8.0) * 2.0 ** (e - 7))
    return np.array(sorted(vals), dtype=f64)


_E4M3 = _e4m3_grid()


def _round_e4m3(y: np.ndarray) -> np.ndarray:
    """Round to the nearest E4M3FN value, ties to even mantissa, saturating
    at +-448.  Returned as float32."""
    y = np.asarray(y, dtype=f64)
    a = np.minimum(np.abs(y), 448.0)
    g = _E4M3
    hi = np.clip(np.searchsorted(g, a, side="left"), 0, len(g) - 1)
    lo = np.clip(hi - 1, 0, len(g) - 1)
    dlo = a - g[lo]
    dhi = g[hi] - a
    # the grid index parity equals the mantissa parity for E4M3
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    r = np.where(pick_hi, g[hi], g[lo])
    r = np.where(a == g[hi], g[hi], r)
    return (np.sign(y) * r).astype(f32)


def quantize_views(x: np.ndarray, fmt: str):
    """Per-view scaled storage: scale_v = max_t |x_v[t]| / Fmax (float32),
    code = round(x / scale_v) in the target format (nearest, ties to even,
    saturating).  The division is done in float32.  Returns (codes as
    float32 values, scale float32 [n])."""
    X = np.asarray(x, dtype=f32)
    amax = np.abs(X).max(axis=1)
    scale = (amax / f32(_FMAX[fmt])).astype(f32)
    scale = np.where(scale == 0, f32(1.0), scale).astype(f32)
    y = (X / scale[:, None]).astype(f32)
    codes = _round_bf16(y) if fmt == "bf16" else _round_e4m3(y)
    return codes, scale


_E2M1 = np.array([0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0], dtype=f64)


def _round_e2m1(y: np.ndarray) -> np.ndarray:
    """Round to the nearest FP4 E2M1 value (ties to even mantissa; grid
    index parity equals mantissa parity), saturating at +-6."""
    y = np.asarray(y, dtype=f64)
    a = np.minimum(np.abs(y), 6.0)
    g = _E2M1
    hi = np.clip(np.searchsorted(g, a, side="left"), 0, len(g) - 1)
    lo = np.clip(hi - 1, 0, len(g) - 1)
    dlo, dhi = a - g[lo], g[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    r = np.where(a == g[hi], g[hi], np.where(pick_hi, g[hi], g[lo]))
    return (np.sign(y) * r).astype(f32)


_MX = {"mxfp8": (8, _round_e4m3), "mxfp4": (2, _round_e2m1)}


def quantize_views_mx(x: np.ndarray, fmt: str):
    """Block-scaled storage with one shared power-of-two scale per 32
    consecutive values of a view (OCP microscaling): the block exponent is
    floor(log2(max |x| of the block)) - emax of the element format (8 for
    e4m3, 2 for e2m1), clamped to [-127, 127] (-127 for an all-zero block),
    stored as E8M0 = exponent + 127; elements are x / 2^exponent rounded to
    the element format (nearest, ties to even, saturating).  Returns (codes
    as float32 values [n, d], e8m0 uint8 [n, d/32])."""
    emax, rnd = _MX[fmt]
    X = np.asarray(x, dtype=f32)
    n, d = X.shape
    blocks = X.reshape(n, d // 32, 32).astype(f64)
    amax = np.abs(blocks).max(axis=2)
    mant, ex = np.frexp(amax)                  # amax = mant * 2^ex, mant in [0.5, 1)
    e = np.where(amax > 0, ex - 1 - emax, -127).clip(-127, 127)
    y = blocks / np.ldexp(1.0, e)[:, :, None]  # exact: division by a power of two
    codes = rnd(y).reshape(n, d)
    return codes, (e + 127).astype(np.uint8)


def dequantize_mx(codes, e8m0):
    c = np.asarray(codes, dtype=f64)
    n, d = c.shape
    scale = np.ldexp(1.0, np.asarray(e8m0, dtype=np.int64) - 127)
    return (c.reshape(n, d // 32, 32) * scale[:, :, None]).reshape(n, d)


def dequantize(codes, scale):
    return np.asarray(codes, dtype=f64) * np.asarray(scale, dtype=f64)[:, None]


def lowprec_exhaustive_scores(qcodes, qscale, qoff, dbcodes, dbscale, n_views,
                              shape_chunk=256):
    """Eq. 3 on the dequantised values: s~ = s_q * s_p * sum_t q~ p~.

    The scales enter each pair before the per-shape max.  float64 (exact
    products of the low-precision codes)."""
    qv = dequantize(qcodes, qscale)
    db = dequantize(dbcodes, dbscale)
    return exhaustive_scores(qv, qoff, db, n_views, f64, shape_chunk)


# --------------------------------------------------------------------------
# Metrics
# --------------------------------------------------------------------------

def recall_at_k(ids_method: np.ndarray, ids_ref: np.ndarray, k: int):
    """Mean and minimum over queries of |T_k(method) & T_k(ref)| / k."""
    r = [len(set(a[:k].tolist()) & set(b[:k].tolist())) / float(k)
         for a, b in zip(ids_method, ids_ref)]
    return float(np.mean(r)), float(np.min(r))
