"""Pins for the CPU oracle: brute force, closed forms, invariants and
library routines that do not share the oracle's code (CPU only)."""
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle as O
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _unit_rows(rng, n, d, nonneg=True):
    x = rng.random((n, d)) if nonneg else rng.standard_normal((n, d))
    x = x / np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(np.float32)


def _tiny(seed=0, N=12, nv=4, d=6, B=3, m=(3, 5)):
    rng = np.random.default_rng(seed)
    db = _unit_rows(rng, N * nv, d)
    counts = rng.integers(m[0], m[1] + 1, size=B)
    qoff = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    q = _unit_rows(rng, int(qoff[-1]), d)
    return q, qoff, db, nv


# ---------------------------------------------------------------- Eq. 3
def test_eq3_matches_scipy_cosine_brute_force():
    q, qoff, db, nv = _tiny()
    S = O.exhaustive_scores(q, qoff, db, nv)
    for b in range(len(qoff) - 1):
        Q = q[qoff[b]:qoff[b + 1]].astype(np.float64)
        for p in range(db.shape[0] // nv):
            P = db[p * nv:(p + 1) * nv].astype(np.float64)
            cos = 1.0 - cdist(Q, P, metric="cosine")
            # float32 rows are unit-norm to ~1e-7, cosine divides the norms out
            assert abs(S[b, p] - cos.max(axis=1).mean()) < 1e-6


def test_eq3_literal_loop_agrees():
    q, qoff, db, nv = _tiny(1, N=5, nv=3, d=4, B=2)
    assert np.allclose(O.exhaustive_scores(q, qoff, db, nv),
                       O.exhaustive_scores_literal(q, qoff, db, nv), atol=1e-13)


def test_eq3_golden_hand_example():
    g = json.load(open(os.path.join(GOLD, "eq3_2d.json")))
    q = np.array(g["query"], np.float32)
    db = np.array(g["db"], np.float32)
    S = O.exhaustive_scores(q, [0, 2], db, g["n_views"])[0]
    assert np.allclose(S, g["S_exhaustive"], atol=1e-7)
    ids, _ = O.rank_topk(S[None], 3)
    assert ids[0].tolist() == g["ranking_top3"]


def test_eq3_single_view_is_plain_cosine():
    rng = np.random.default_rng(3)
    db = _unit_rows(rng, 10, 7, nonneg=False)
    q = _unit_rows(rng, 1, 7, nonneg=False)
    S = O.exhaustive_scores(q, [0, 1], db, 1)[0]
    cos = 1.0 - cdist(q.astype(np.float64), db.astype(np.float64), "cosine")[0]
    assert np.allclose(S, cos, atol=1e-6)


def test_eq3_self_score_one_and_maximal_and_bounded():
    w = synth.PRESETS["c1"].scaled(n_shapes=60, dim=32, n_queries=2)
    db, _, _ = synth.make_db(w)
    nv = w.n_views
    sel = [5, 17, 42]
    q = np.concatenate([db[s * nv:(s + 1) * nv] for s in sel])
    qoff = np.arange(len(sel) + 1, dtype=np.int32) * nv
    S = O.exhaustive_scores(q, qoff, db, nv)
    for b, s in enumerate(sel):
        assert abs(S[b, s] - 1.0) < 1e-6
        assert S[b, s] >= S[b].max() - 1e-6
        assert O.rank_topk(S[b:b + 1], 1)[0][0, 0] == s
    assert S.min() >= 0.0 and S.max() <= 1.0 + 1e-6


def test_eq3_permutation_invariance():
    q, qoff, db, nv = _tiny(4, N=8, nv=5, d=8, B=2)
    S = O.exhaustive_scores(q, qoff, db, nv)
    rng = np.random.default_rng(0)
    db2 = db.copy()
    for p in range(db.shape[0] // nv):
        db2[p * nv:(p + 1) * nv] = db[p * nv + rng.permutation(nv)]
    assert np.array_equal(S, O.exhaustive_scores(q, qoff, db2, nv))
    q2 = q.copy()
    for b in range(len(qoff) - 1):
        lo, hi = qoff[b], qoff[b + 1]
        q2[lo:hi] = q[lo + rng.permutation(hi - lo)]
    assert np.allclose(S, O.exhaustive_scores(q2, qoff, db, nv), atol=1e-14)


# ---------------------------------------------------------------- ranking
def test_rank_matches_python_sorted():
    rng = np.random.default_rng(5)
    s = np.round(rng.random((3, 40)), 1)  # many exact ties
    ids, vals = O.rank_topk(s, 15)
    for b in range(3):
        ref = sorted(range(40), key=lambda i: (-s[b, i], i))[:15]
        assert ids[b].tolist() == ref
        assert np.array_equal(vals[b], s[b, ref])


# ---------------------------------------------------------------- quantizer
def test_quantizer_brute_force_and_forms():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((30, 5)).astype(np.float32)
    B = rng.standard_normal((9, 5)).astype(np.float32)
    a = O.assign(x, B, 3)
    for n in range(30):
        d = [sum((float(x[n, t]) - float(B[k, t])) ** 2 for t in range(5)) for k in range(9)]
        ref = sorted(range(9), key=lambda k: (d[k], k))[:3]
        assert a[n].tolist() == ref
    assert np.allclose(O.quantizer_dist(x, B), O.quantizer_dist(x, B, direct=True), atol=1e-12)


def test_quantizer_ties_go_to_lowest_index():
    B = np.array([[0, 1], [1, 0], [0, 1], [1, 0]], np.float32)
    x = np.array([[0.1, 0.9], [0.9, 0.1], [0.5, 0.5]], np.float32)
    assert O.assign(x, B, 1)[:, 0].tolist() == [0, 1, 0]
    assert O.assign(x, B, 2).tolist() == [[0, 2], [1, 3], [0, 1]]


# ---------------------------------------------------------------- k-means
def test_kmeans_matches_sklearn_lloyd():
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(7)
    cent = rng.standard_normal((6, 8)) * 4
    X = (cent[rng.integers(0, 6, 600)] + rng.standard_normal((600, 8))).astype(np.float32)
    init = synth.kmeans_init_idx(600, 6, 11)
    B, a, it = O.kmeans(X, init, 50)
    km = KMeans(6, init=X[init].astype(np.float64), n_init=1, algorithm="lloyd",
                tol=0.0, max_iter=50).fit(X.astype(np.float64))
    assert np.array_equal(a, km.labels_)
    assert np.allclose(B, km.cluster_centers_, atol=1e-5)


def test_kmeans_separated_blobs_closed_form():
    rng = np.random.default_rng(8)
    blobs = [np.array([10.0, 0]), np.array([-10.0, 0]), np.array([0, 10.0])]
    X = np.concatenate([c + 0.1 * rng.standard_normal((20, 2)) for c in blobs]).astype(np.float32)
    B, a, it = O.kmeans(X, np.array([0, 20, 40]), 25)
    assert it == 1  # one update reaches the fixed point; the reassignment confirms it
    for k in range(3):
        assert np.allclose(B[k], X[20 * k:20 * (k + 1)].astype(np.float64).mean(0), atol=1e-6)
        assert (a[20 * k:20 * (k + 1)] == k).all()


def test_kmeans_objective_never_increases():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((400, 4)).astype(np.float32)
    init = synth.kmeans_init_idx(400, 12, 3)
    prev = np.inf
    for t in range(1, 8):
        B, a, _ = O.kmeans(X, init, t)
        obj = float(((X.astype(np.float64) - B[a].astype(np.float64)) ** 2).sum())
        assert obj <= prev + 1e-9
        prev = obj


# ---------------------------------------------------------------- F-IF
def test_build_fif_structure_brute_force():
    q, qoff, db, nv = _tiny(10, N=10, nv=4, d=6)
    rng = np.random.default_rng(1)
    K = 5
    B = _unit_rows(rng, K, 6)
    for ma in (1, 2, 3):
        W = O.assign(db, B, ma)
        off, es, ev = O.build_fif(W, K, nv)
        assert off[-1] == ma * db.shape[0]
        for w in range(K):
            lst = list(zip(es[off[w]:off[w + 1]].tolist(), ev[off[w]:off[w + 1]].tolist()))
            assert lst == sorted(lst)
            ref = [(v // nv, v % nv) for v in range(db.shape[0]) if w in W[v].tolist()]
            assert lst == ref


def _fif(q, qoff, db, nv, B, ma):
    W = O.assign(db, B, ma)
    off, es, ev = O.build_fif(W, B.shape[0], nv)
    return O.fif_scores(q, qoff, db, nv, B, off, es, ev), W


def test_eq4_list_form_equals_literal_delta_form():
    q, qoff, db, nv = _tiny(11, N=7, nv=3, d=5, B=2)
    rng = np.random.default_rng(2)
    B = _unit_rows(rng, 4, 5)
    for ma in (1, 2):
        S, W = _fif(q, qoff, db, nv, B, ma)
        L = O.fif_scores_literal(q, qoff, db, nv, B, W)
        assert np.allclose(S, L, atol=1e-13)


def test_eq4_golden_hand_example():
    g = json.load(open(os.path.join(GOLD, "eq3_2d.json")))
    q = np.array(g["query"], np.float32)
    db = np.array(g["db"], np.float32)
    B = np.array(g["codebook"], np.float32)
    S, _ = _fif(q, np.array([0, 2]), db, g["n_views"], B, 1)
    assert np.allclose(S[0], g["S_fif"], atol=1e-7)


def test_eq4_reduces_to_eq3_for_one_word_and_full_ma():
    q, qoff, db, nv = _tiny(12, N=9, nv=4, d=6)
    S3 = O.exhaustive_scores(q, qoff, db, nv)
    rng = np.random.default_rng(3)
    S1, _ = _fif(q, qoff, db, nv, _unit_rows(rng, 1, 6), 1)
    assert np.allclose(S1, S3, atol=1e-13)
    B = _unit_rows(rng, 5, 6)
    SK, _ = _fif(q, qoff, db, nv, B, 5)
    assert np.allclose(SK, S3, atol=1e-13)


def test_eq4_bounded_by_eq3_and_monotone_in_ma():
    q, qoff, db, nv = _tiny(13, N=20, nv=6, d=8, B=4)
    S3 = O.exhaustive_scores(q, qoff, db, nv)
    rng = np.random.default_rng(4)
    B = _unit_rows(rng, 6, 8)
    prev = None
    for ma in range(1, 7):
        S, _ = _fif(q, qoff, db, nv, B, ma)
        assert (S >= 0).all() and (S <= S3 + 1e-12).all()
        if prev is not None:
            assert (S >= prev - 1e-12).all()
        prev = S


# ---------------------------------------------------------------- S-IF
def test_sif_golden_hand_example():
    g = json.load(open(os.path.join(GOLD, "sif_4shape.json")))
    ids = np.array(g["nbr_ids"])
    sc = np.array(g["nbr_scores"])
    l1, po, pid, pv = O.build_sif(ids, sc, g["n_shapes"])
    assert np.allclose(l1, g["l1"])
    for i, lst in g["postings"].items():
        i = int(i)
        got = list(zip(pid[po[i]:po[i + 1]].tolist(), pv[po[i]:po[i + 1]].tolist()))
        assert [(a, pytest.approx(b)) for a, b in lst] == got
    for p in range(4):
        _, _, S = O.rerank_sif(l1, po, pid, pv, ids[p], sc[p], 0.0, 4)
        assert np.allclose(S, g["S_prime"][p], atol=1e-12)


def _random_nbrs(rng, N, k1):
    ids = np.empty((N, k1), np.int64)
    sc = np.empty((N, k1))
    for p in range(N):
        others = rng.choice([i for i in range(N) if i != p], size=k1 - 1, replace=False)
        ids[p] = [p] + others.tolist()
        sc[p] = [1.0] + sorted(rng.random(k1 - 1).tolist(), reverse=True)
    return ids, sc


def test_sif_inverted_equals_dense_eq8():
    rng = np.random.default_rng(14)
    N, k1 = 30, 6
    ids, sc = _random_nbrs(rng, N, k1)
    l1, po, pid, pv = O.build_sif(ids, sc, N)
    for p in range(N):
        _, _, S = O.rerank_sif(l1, po, pid, pv, ids[p], sc[p], 0.0, N)
        D = O.rerank_sif_dense(ids, sc, ids[p], sc[p], 0.0, N)
        assert np.allclose(S, D, atol=1e-12)
    # an outside query with a virtual self membership
    qi = rng.choice(N, size=k1 - 1, replace=False)
    qs = rng.random(k1 - 1)
    _, _, S = O.rerank_sif(l1, po, pid, pv, qi, qs, 1.0, N)
    D = O.rerank_sif_dense(ids, sc, qi, qs, 1.0, N)
    assert np.allclose(S, D, atol=1e-12)


def test_sif_crisp_memberships_give_set_jaccard_eq5():
    rng = np.random.default_rng(15)
    N, k1 = 25, 5
    ids, _ = _random_nbrs(rng, N, k1)
    ones = np.ones(ids.shape)
    l1, po, pid, pv = O.build_sif(ids, ones, N)
    for q in range(N):
        _, _, S = O.rerank_sif(l1, po, pid, pv, ids[q], ones[q], 0.0, N)
        for p in range(N):
            a, b = set(ids[q].tolist()), set(ids[p].tolist())
            assert abs(S[p] - len(a & b) / len(a | b)) < 1e-12


def test_sif_self_one_symmetric_bounded():
    rng = np.random.default_rng(16)
    N, k1 = 20, 4
    ids, sc = _random_nbrs(rng, N, k1)
    l1, po, pid, pv = O.build_sif(ids, sc, N)
    M = np.stack([O.rerank_sif(l1, po, pid, pv, ids[p], sc[p], 0.0, N)[2] for p in range(N)])
    assert np.allclose(np.diag(M), 1.0)
    assert np.allclose(M, M.T, atol=1e-12)
    assert M.min() >= 0 and M.max() <= 1 + 1e-12


def test_neighbour_augment_k2_one_is_identity():
    rng = np.random.default_rng(17)
    N, k1 = 10, 4
    ids, sc = _random_nbrs(rng, N, k1)
    F = np.zeros((N, N))
    for p in range(N):
        F[p, ids[p]] = sc[p]
    assert np.array_equal(O.neighbour_augment(F, ids, 1), F)
    F2 = O.neighbour_augment(F, ids, 2)
    assert np.allclose(F2[0], (F[0] + F[ids[0, 1]]) / 2)


# ---------------------------------------------------------------- precision
def test_bf16_quantizer_matches_torch_cast():
    import torch
    rng = np.random.default_rng(18)
    x = _unit_rows(rng, 64, 100)
    codes, scale = O.quantize_views(x, "bf16")
    y = torch.from_numpy(x) / torch.from_numpy(scale)[:, None]
    ref = y.to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(codes, ref)
    assert np.array_equal(scale, np.abs(x).max(1))


def test_fp8_quantizer_matches_torch_cast():
    import torch
    rng = np.random.default_rng(19)
    x = _unit_rows(rng, 64, 100)
    codes, scale = O.quantize_views(x, "fp8")
    y = (torch.from_numpy(x) / torch.from_numpy(scale)[:, None]).clamp(-448, 448)
    ref = y.to(torch.float8_e4m3fn).to(torch.float32).numpy()
    assert np.array_equal(codes, ref)
    # every code lies on the E4M3 grid and the view maximum maps to 448
    assert np.allclose(np.abs(codes).max(1), 448.0)
    # grid spot checks: ties to even mantissa and subnormals
    t = np.array([[1.0625, 1.1875, 2.0 ** -9, 2.0 ** -10, 300.0, 460.0, 0.013671875]], np.float32)
    from oracle.gift_oracle import _round_e4m3
    c = _round_e4m3(t)
    assert c.tolist() == [[1.0, 1.25, 2.0 ** -9, 0.0, 288.0, 448.0, 0.013671875]]


def test_lowprec_scores_close_to_fp64():
    w = synth.PRESETS["c1"].scaled(n_shapes=50, dim=64, n_queries=3)
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    S = O.exhaustive_scores(q, qoff, db, w.n_views)
    for fmt, tol in (("bf16", 8e-3), ("fp8", 0.13)):
        qc, qs = O.quantize_views(q, fmt)
        dc, ds = O.quantize_views(db, fmt)
        L = O.lowprec_exhaustive_scores(qc, qs, qoff, dc, ds, w.n_views)
        assert np.abs(L - S).max() < tol


def test_recall_metric():
    a = np.array([[1, 2, 3, 4]])
    b = np.array([[4, 3, 9, 8]])
    assert O.recall_at_k(a, b, 4) == (0.5, 0.5)


# ---------------------------------------------------------------- Eq. 9 / 11
def test_fusion_generalised_mean_closed_forms():
    rng = np.random.default_rng(22)
    a = rng.random(50)
    b = rng.random(50)
    # alpha = 1 is the arithmetic mean
    assert np.allclose(O.fuse_activations(a, b, 1.0), (a + b) / 2)
    # equal inputs are a fixed point for any alpha
    assert np.allclose(O.fuse_activations(a, a, 0.5), a)
    # alpha = 0.5 written out: ((sqrt a + sqrt b) / 2)^2
    assert np.allclose(O.fuse_activations(a, b, 0.5), ((np.sqrt(a) + np.sqrt(b)) / 2) ** 2)
    # one side zero: a / 2^(1/alpha)
    assert np.allclose(O.fuse_activations(a, np.zeros(50), 0.5), a / 4)
    # the generalised mean lies between min and max and grows with alpha
    lo = O.fuse_activations(a, b, 0.5)
    hi = O.fuse_activations(a, b, 1.0)
    assert (lo <= hi + 1e-15).all()
    assert (lo >= np.minimum(a, b) - 1e-15).all() and (hi <= np.maximum(a, b) + 1e-15).all()


def test_co_augmentation_swaps_neighbour_sets():
    rng = np.random.default_rng(23)
    N = 12
    F1 = rng.random((N, N))
    F2 = rng.random((N, N))
    n1 = np.stack([np.concatenate([[p], rng.permutation(np.delete(np.arange(N), p))])
                   for p in range(N)])
    n2 = np.stack([np.concatenate([[p], rng.permutation(np.delete(np.arange(N), p))])
                   for p in range(N)])
    A1, A2 = O.co_augment(F1, F2, n1, n2, 3)
    for p in range(N):
        assert np.allclose(A1[p], F1[n2[p, :3]].mean(0))
        assert np.allclose(A2[p], F2[n1[p, :3]].mean(0))


# ---------------------------------------------------------------- MX storage
def test_mx_element_rounding_hand_cases():
    from oracle.gift_oracle import _round_e2m1
    t = np.array([0.25, 0.75, 1.25, 1.75, 2.5, 3.5, 5.0, 7.0, -2.6, 0.2], np.float32)
    # ties to even mantissa: 0.25 -> 0, 0.75 -> 1.0, 1.25 -> 1.0, 1.75 -> 2.0,
    # 2.5 -> 2.0, 3.5 -> 4.0, 5.0 -> 4.0; saturation 7 -> 6
    assert _round_e2m1(t).tolist() == [0.0, 1.0, 1.0, 2.0, 2.0, 4.0, 4.0, 6.0, -3.0, 0.0]


def test_mx_block_scales_and_error():
    rng = np.random.default_rng(30)
    x = (rng.random((20, 128)) ** 2).astype(np.float32)
    x[3, :32] = 0.0                      # an all-zero block
    x[4, 32:64] = 2.0 ** -5              # a power-of-two block
    for fmt, emax, rel in (("mxfp8", 8, 2.0 ** -3), ("mxfp4", 2, 2.0 ** -1)):
        codes, e = O.quantize_views_mx(x, fmt)
        assert e.shape == (20, 4) and e.dtype == np.uint8
        assert e[3, 0] == 0 and np.all(codes[3, :32] == 0)
        # a block of 2^-5 has exponent -5 - emax, and codes 2^emax
        assert e[4, 1] == 127 - 5 - emax
        assert np.all(codes[4, 32:64] == 2.0 ** emax)
        # largest code of a non-zero block lies in [2^emax, 2^(emax+1)]
        blk = np.abs(codes.reshape(20, 4, 32)).max(axis=2)
        nz = blk > 0
        assert (blk[nz] >= 2.0 ** emax).all() and (blk[nz] <= 2.0 ** (emax + 1)).all()
        # element error within half a step of the format relative to the block max
        deq = O.dequantize_mx(codes, e)
        bmax = np.abs(x.reshape(20, 4, 32)).max(axis=2, keepdims=True)
        err = np.abs(deq.reshape(20, 4, 32) - x.reshape(20, 4, 32))
        assert (err <= rel * bmax + 1e-30).all()
