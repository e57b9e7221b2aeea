"""GPU parity of the first inverted file (Sec. 2.3, Eq. 4) against the
CPU oracle: quantizer words, k-means codebooks, lists and ranked ids."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth
from test_gpu_exhaustive import (REL, assert_flags_as_predicted, assert_ranked_equal,
                                 assert_returned_exact)

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1604_01879_amd import _lib
    return _lib


def _wl(**kw):
    base = dict(n_shapes=200, dim=128, n_queries=5, m_lo=64, m_hi=64, p_dis=0.2)
    base.update(kw)
    return synth.PRESETS["c1"].scaled(**base)


def _assert_words(words, x, cb, ma):
    """GPU words equal the oracle's; a difference is allowed only between
    codewords whose float64 distances tie to 1e-12."""
    ref = O.assign(x, cb, ma)
    if np.array_equal(words, ref):
        return
    d = O.quantizer_dist(x, cb)
    bad = np.flatnonzero((words != ref).any(axis=1))
    for r in bad:
        assert np.allclose(d[r, words[r]], d[r, ref[r]], atol=1e-12, rtol=0), (r, words[r], ref[r])


@pytest.mark.parametrize("ma", [1, 3])
def test_assign_matches_oracle(L, ma):
    _say(f"assign ma={ma}")
    w = _wl()
    db, _, _ = synth.make_db(w)
    x = db[:3000]
    cb = db[synth.kmeans_init_idx(db.shape[0], 50, 1)]
    words, unc = L.gift_assign(torch.from_numpy(x).to(DEV), torch.from_numpy(cb).to(DEV), ma)
    torch.cuda.synchronize()
    assert int(unc.item()) == 0
    _assert_words(words.cpu().numpy(), x, cb, ma)


@pytest.mark.parametrize("dim", [32, 64, 96, 192, 256])
@pytest.mark.parametrize("ma", [1, 3])
def test_assign_row_lengths(L, dim, ma):
    """The quantizer (pipelined GEMM on BF16-split rows) against the oracle
    for rows of 1, 2, 3, 6 and 8 sub-tiles of 32 values, so the two LDS
    stages end on either parity, with ragged 256 x 256 tiles (1,000 rows,
    300 codewords)."""
    _say(f"assign dim={dim} ma={ma}")
    w = _wl(n_shapes=40, dim=dim, n_views=25)
    db, _, _ = synth.make_db(w)
    x = db[:1000]
    cb = db[synth.kmeans_init_idx(db.shape[0], 300, 6)]
    words, unc = L.gift_assign(torch.from_numpy(x).to(DEV), torch.from_numpy(cb).to(DEV), ma)
    torch.cuda.synchronize()
    assert int(unc.item()) == 0
    _assert_words(words.cpu().numpy(), x, cb, ma)


def test_assign_duplicate_codewords_go_to_lowest_index(L):
    _say("assign duplicates")
    rng = np.random.default_rng(2)
    base = rng.random((6, 64)).astype(np.float32)
    cb = np.concatenate([base, base[::-1], base]).astype(np.float32)  # every codeword 3x
    x = (base[rng.integers(0, 6, 200)] + 0.01 * rng.random((200, 64))).astype(np.float32)
    words, _ = L.gift_assign(torch.from_numpy(x).to(DEV), torch.from_numpy(cb).to(DEV), 3)
    words = words.cpu().numpy()
    ref = O.assign(x, cb, 3)
    assert np.array_equal(words, ref)
    # the three copies of the nearest vector, lowest index first
    assert (words[:, 0] < 6).all()


def test_build_codebook_bit_exact(L):
    _say("k-means")
    w = _wl(n_shapes=60, dim=64, n_classes=10)
    db, _, _ = synth.make_db(w)
    K = 24
    init = synth.kmeans_init_idx(db.shape[0], K, 5)
    B, a, it = O.kmeans(db, init, 25)
    cb, ag, itg = L.gift_build_codebook(torch.from_numpy(db).to(DEV), K, init, 25)
    torch.cuda.synchronize()
    assert itg == it
    assert np.array_equal(ag.cpu().numpy(), a)
    assert np.array_equal(cb.cpu().numpy(), B)


def test_build_codebook_capped_iterations(L):
    _say("k-means capped")
    w = _wl(n_shapes=40, dim=64, n_classes=8)
    db, _, _ = synth.make_db(w)
    init = synth.kmeans_init_idx(db.shape[0], 16, 9)
    for t in (0, 1, 2):
        B, a, it = O.kmeans(db, init, t)
        cb, ag, itg = L.gift_build_codebook(torch.from_numpy(db).to(DEV), 16, init, t)
        assert itg == it
        assert np.array_equal(cb.cpu().numpy(), B)
        assert np.array_equal(ag.cpu().numpy(), a)


@pytest.mark.parametrize("ma", [1, 2, 3])
def test_build_fif_bit_exact(L, ma):
    _say(f"build_fif ma={ma}")
    w = _wl(n_shapes=90, dim=96, n_views=37)
    db, _, _ = synth.make_db(w)
    cb = db[synth.kmeans_init_idx(db.shape[0], 20, 3)]
    V = L.Views(torch.from_numpy(db).to(DEV), w.n_views, L.F32)
    F = L.gift_build_fif(V, torch.from_numpy(cb).to(DEV), ma)
    torch.cuda.synchronize()
    W = O.assign(db, cb, ma)
    off, es, ev = O.build_fif(W, 20, w.n_views)
    assert np.array_equal(F.view_words.cpu().numpy(), W)
    assert np.array_equal(F.offsets.cpu().numpy(), off)
    assert np.array_equal(F.entry_shape.cpu().numpy(), es)
    assert np.array_equal(F.entry_view.cpu().numpy(), ev)


def _fif_case(L, w, K, ma, dtype):
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    cb = db[synth.kmeans_init_idx(db.shape[0], K, 4)]
    master = torch.from_numpy(db).to(DEV)
    V32 = L.Views(master, w.n_views, L.F32)
    F = L.gift_build_fif(V32, torch.from_numpy(cb).to(DEV), ma)
    if dtype == L.F32:
        V = V32
    else:
        codes, scale = L.gift_quantize_views(master, dtype)
        V = L.Views(codes, w.n_views, dtype, scale, master)
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    W = O.assign(db, cb, ma)
    off, es, ev = O.build_fif(W, K, w.n_views)
    return db, q, qoff, cb, V, F, Q, (off, es, ev)


@pytest.mark.parametrize("dtype_name", ["f32", "bf16", "fp8"])
def test_first_pass_fif_scores(L, dtype_name):
    _say(f"fif first pass {dtype_name}")
    dt = {"f32": L.F32, "bf16": L.BF16, "fp8": L.FP8E4M3}[dtype_name]
    w = _wl(n_shapes=150, dim=128, m_lo=1, m_hi=64)
    db, q, qoff, cb, V, F, Q, (off, es, ev) = _fif_case(L, w, 12, 2, dt)
    S, qw = L.gift_score_fif(V, F, Q)
    torch.cuda.synchronize()
    qw = qw.cpu().numpy()
    assert np.array_equal(qw, O.assign(q, cb, 1)[:, 0])
    if dtype_name == "f32":
        ref = O.fif_scores(q, qoff, db, w.n_views, cb, off, es, ev)
    else:
        qc, qs = O.quantize_views(q, dtype_name)
        dc, ds = O.quantize_views(db, dtype_name)
        ref = O.fif_scores(O.dequantize(qc, qs), qoff, O.dequantize(dc, ds), w.n_views, cb,
                           off, es, ev, qwords=qw)
    assert np.allclose(S.cpu().numpy(), ref, rtol=REL, atol=1e-6)


@pytest.mark.parametrize("dtype_name", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("n_group", [1, 15, 16, 17, 31, 32, 33, 130])
@pytest.mark.parametrize("dim", [96, 256])
def test_scan_group_sizes_around_narrow_tile(L, dtype_name, n_group, dim):
    """One word (K = 1) puts every query view of the batch in one group: up
    to 16 views take the 128 x 16 scan tile (float32 rows of whole 128-byte
    sub-tiles), up to 32 the 128 x 32 tile, more the 128 x 128 tiles (130
    views: two column passes, the second of 2 views).  float32 rows of 384
    and 1,024 bytes and BF16 rows of 512 bytes take the direct-to-LDS narrow
    loop, e4m3 rows of 96 bytes the register-staged one, BF16 rows of 192
    bytes the 128 x 128 tiles."""
    _say(f"fif group of {n_group} {dtype_name} dim {dim}")
    dt = {"f32": L.F32, "bf16": L.BF16, "fp8": L.FP8E4M3}[dtype_name]
    w = _wl(n_shapes=70, dim=dim, n_queries=1, m_lo=n_group, m_hi=n_group, n_views=19)
    db, q, qoff, cb, V, F, Q, (off, es, ev) = _fif_case(L, w, 1, 1, dt)
    S, qw = L.gift_score_fif(V, F, Q)
    torch.cuda.synchronize()
    assert int(qoff[-1]) == n_group and (qw.cpu().numpy() == 0).all()
    if dtype_name == "f32":
        ref = O.fif_scores(q, qoff, db, w.n_views, cb, off, es, ev)
    else:
        qc, qs = O.quantize_views(q, dtype_name)
        dc, ds = O.quantize_views(db, dtype_name)
        ref = O.fif_scores(O.dequantize(qc, qs), qoff, O.dequantize(dc, ds), w.n_views, cb,
                           off, es, ev, qwords=qw.cpu().numpy())
    assert np.allclose(S.cpu().numpy(), ref, rtol=REL, atol=1e-6)


@pytest.mark.parametrize("fmt", ["mxfp8", "mxfp4"])
def test_first_pass_fif_scores_mx(L, fmt):
    """MX block-scaled list payloads: the first pass equals Eq. 4 over the
    dequantised MX views (words decided on the float32 views)."""
    _say(f"fif first pass {fmt}")
    dt = L.MXFP8 if fmt == "mxfp8" else L.MXFP4
    w = _wl(n_shapes=150, dim=256, m_lo=1, m_hi=64)
    db, q, qoff, cb, V, F, Q, (off, es, ev) = _fif_case(L, w, 12, 2, dt)
    S, qw = L.gift_score_fif(V, F, Q)
    torch.cuda.synchronize()
    qw = qw.cpu().numpy()
    assert np.array_equal(qw, O.assign(q, cb, 1)[:, 0])
    qc, qe = O.quantize_views_mx(q, fmt)
    dc, de = O.quantize_views_mx(db, fmt)
    ref = O.fif_scores(O.dequantize_mx(qc, qe), qoff, O.dequantize_mx(dc, de), w.n_views, cb,
                       off, es, ev, qwords=qw)
    assert np.allclose(S.cpu().numpy(), ref, rtol=REL, atol=1e-6)


@pytest.mark.parametrize("fmt", ["mxfp8", "mxfp4"])
def test_query_fif_mx_rescored_all(L, fmt):
    """With every shape rescored from the float32 master, the MX path's
    ranking is the exact Eq. 4 ranking."""
    _say(f"query_fif {fmt} full rescore")
    dt = L.MXFP8 if fmt == "mxfp8" else L.MXFP4
    w = _wl(n_shapes=240, dim=256, m_lo=4, m_hi=64, n_queries=5)
    db, q, qoff, cb, V, F, Q, (off, es, ev) = _fif_case(L, w, 16, 2, dt)
    k = 20
    ids, sc, flags = L.gift_query_fif(V, F, Q, k, w.n_shapes)
    torch.cuda.synchronize()
    S = O.fif_scores(q, qoff, db, w.n_views, cb, off, es, ev)
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    for b in range(len(qoff) - 1):
        assert_ranked_equal(ids[b], sc[b], S[b], k)
    assert (flags.cpu().numpy() & 1).all()  # every shape was rescored


@pytest.mark.parametrize("dtype_name", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("ma", [1, 3])
@pytest.mark.parametrize("R", [300, 120, 60])
def test_query_fif_ranked_ids(L, dtype_name, ma, R):
    """Eq. 4 ranking with every shape rescored (R = N) and with the top 120 or
    60 of 300: returned scores are the exact Eq. 4 scores of their ids in
    (score desc, id asc) order on every row; a certified row is the exact
    top k; the certificate holds where the oracle's first pass leaves it
    room (e4m3 at R = 60: only where its margin is positive)."""
    _say(f"query_fif {dtype_name} ma={ma} R={R}")
    dt = {"f32": L.F32, "bf16": L.BF16, "fp8": L.FP8E4M3}[dtype_name]
    w = _wl(n_shapes=300, dim=128, m_lo=4, m_hi=64, n_queries=6)
    db, q, qoff, cb, V, F, Q, (off, es, ev) = _fif_case(L, w, 16, ma, dt)
    k = 20
    ids, sc, flags = L.gift_query_fif(V, F, Q, k, R)
    torch.cuda.synchronize()
    S = O.fif_scores(q, qoff, db, w.n_views, cb, off, es, ev)
    ids, sc, flags = ids.cpu().numpy(), sc.cpu().numpy(), flags.cpu().numpy()
    if dtype_name == "f32":
        S1 = S
    else:
        qc, qs = O.quantize_views(q, dtype_name)
        dc, ds = O.quantize_views(db, dtype_name)
        S1 = O.fif_scores(O.dequantize(qc, qs), qoff, O.dequantize(dc, ds), w.n_views, cb,
                          off, es, ev, qwords=O.assign(q, cb, 1)[:, 0])
    for b in range(len(qoff) - 1):
        assert_returned_exact(ids[b], sc[b], S[b], k)
        if dtype_name == "f32" or R == w.n_shapes or flags[b] & 1:
            assert_ranked_equal(ids[b], sc[b], S[b], k)
    need = assert_flags_as_predicted(flags, S1, S, qoff, R, k, dtype_name, w.dim,
                                     list_scan=True)
    assert (flags >> 1 == 0).all()  # every query word certified
    if R == w.n_shapes:
        assert (flags == 1).all()
    if not (dtype_name == "fp8" and R == 60 and ma == 3):
        assert need >= 1


def test_query_fif_long_rows_zero_ties(L):
    """Rows of 40,000 shapes with a large vocabulary, so each query matches
    a few hundred shapes and the rest score 0: the chunked top-r selection
    resolves the tie at 0 by id in every chunk and in the merge, and the
    returned tail is the lowest-id zero-score shapes."""
    _say("fif long rows")
    w = _wl(n_shapes=40000, dim=32, n_views=1, m_lo=2, m_hi=4, n_queries=3)
    db, q, qoff, cb, V, F, Q, (off, es, ev) = _fif_case(L, w, 1000, 1, L.F32)
    k, R = 250, 256
    ids, sc, flags = L.gift_query_fif(V, F, Q, k, R)
    torch.cuda.synchronize()
    S = O.fif_scores(q, qoff, db, w.n_views, cb, off, es, ev)
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    for b in range(len(qoff) - 1):
        assert (S[b] > 0).sum() < k  # the tail is zero-score shapes
        assert_ranked_equal(ids[b], sc[b], S[b], k)
        ref_ids, _ = O.rank_topk(S[b][None], k)
        zero = S[b][ref_ids[0]] == 0
        assert np.array_equal(ids[b][zero], ref_ids[0][zero])  # zero ties in id order


@pytest.mark.parametrize("ma", [1, 2])
def test_query_fif_shared_candidates(L, ma):
    """Eq. 4 ranking when every query rescores every shape (each candidate
    shared by all queries, word-matched view pairs), queries of 10..140
    views."""
    _say(f"fif shared candidates ma={ma}")
    w = _wl(n_shapes=37, dim=96, m_lo=10, m_hi=140, n_queries=5)
    db, q, qoff, cb, V, F, Q, (off, es, ev) = _fif_case(L, w, 9, ma, L.F32)
    k, R = 14, 37
    ids, sc, flags = L.gift_query_fif(V, F, Q, k, R)
    torch.cuda.synchronize()
    S = O.fif_scores(q, qoff, db, w.n_views, cb, off, es, ev)
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    for b in range(len(qoff) - 1):
        assert_ranked_equal(ids[b], sc[b], S[b], k)


@pytest.mark.parametrize("dtype_name", ["f32", "bf16"])
def test_query_fif_shared_candidates_batch_equals_single_queries(L, dtype_name):
    """Eq. 4 ranking of a 16-query batch whose candidates repeat against each
    query alone: identical ids, scores and flags, and the oracle's ranking.
    Queries of 1..150 views."""
    _say(f"fif shared-candidate batch {dtype_name}")
    dt = {"f32": L.F32, "bf16": L.BF16}[dtype_name]
    w = _wl(n_shapes=240, dim=128, m_lo=1, m_hi=150, n_queries=16)
    db, q, qoff, cb, V, F, Q, (off, es, ev) = _fif_case(L, w, 12, 2, dt)
    k, R = 12, 50
    ids, sc, fl = L.gift_query_fif(V, F, Q, k, R)
    torch.cuda.synchronize()
    ids, sc, fl = ids.cpu().numpy(), sc.cpu().numpy(), fl.cpu().numpy()
    S = O.fif_scores(q, qoff, db, w.n_views, cb, off, es, ev)
    assert (fl >> 1 == 0).all()  # every query word certified
    for b in range(len(qoff) - 1):
        lo, hi = qoff[b], qoff[b + 1]
        qo = np.array([0, hi - lo], np.int32)
        Q1 = L.Queries(torch.from_numpy(q[lo:hi]).to(DEV), torch.from_numpy(qo))
        i1, s1, f1 = L.gift_query_fif(V, F, Q1, k, R)
        assert np.array_equal(i1.cpu().numpy()[0], ids[b])
        assert np.array_equal(s1.cpu().numpy()[0], sc[b])
        assert int(f1.cpu().numpy()[0]) == int(fl[b])
        assert_returned_exact(ids[b], sc[b], S[b], k)
        if dtype_name == "f32" or fl[b] & 1:
            assert_ranked_equal(ids[b], sc[b], S[b], k)


def test_fif_one_word_and_full_ma_equal_exhaustive(L):
    """K = 1 and MA = K both make Eq. 4 identical to Eq. 3."""
    _say("fif reduces to exhaustive")
    w = _wl(n_shapes=160, dim=64, m_lo=3, m_hi=64)
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    master = torch.from_numpy(db).to(DEV)
    V = L.Views(master, w.n_views, L.F32)
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    ids0, sc0, _ = L.gift_query_exhaustive(V, Q, 15, 60)
    for K, ma in ((1, 1), (4, 4)):
        cb = db[synth.kmeans_init_idx(db.shape[0], K, 2)]
        F = L.gift_build_fif(V, torch.from_numpy(cb).to(DEV), ma)
        ids1, sc1, _ = L.gift_query_fif(V, F, Q, 15, 60)
        assert np.array_equal(ids0.cpu().numpy(), ids1.cpu().numpy())
        assert np.array_equal(sc0.cpu().numpy(), sc1.cpu().numpy())


def test_config1_end_to_end(L):
    """The CPU-sized configuration end to end: 1,000 shapes x 64 views x 256-d,
    40 classes, 8 queries x 64 views, 64-word k-means codebook over all
    database views, MA in {1, 2}, top-10: codebook, assignments, lists and
    ranked ids bit-exact against the oracle."""
    _say("config 1 end to end")
    w = synth.PRESETS["c1"]
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    init = synth.kmeans_init_idx(db.shape[0], w.K, w.seed)
    B, a, it = O.kmeans(db, init, 25)
    master = torch.from_numpy(db).to(DEV)
    cb, ag, itg = L.gift_build_codebook(master, w.K, init, 25)
    assert itg == it and np.array_equal(ag.cpu().numpy(), a)
    assert np.array_equal(cb.cpu().numpy(), B)
    V = L.Views(master, w.n_views, L.F32)
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    S3 = O.exhaustive_scores(q, qoff, db, w.n_views)
    ids, sc, fl = L.gift_query_exhaustive(V, Q, w.top_k, 64)
    for b in range(w.n_queries):
        assert_ranked_equal(ids.cpu().numpy()[b], sc.cpu().numpy()[b], S3[b], w.top_k)
    assert fl.cpu().numpy().all()
    for ma in w.ma:
        F = L.gift_build_fif(V, cb, ma)
        W = O.assign(db, B, ma)
        off, es, ev = O.build_fif(W, w.K, w.n_views)
        assert np.array_equal(F.offsets.cpu().numpy(), off)
        assert np.array_equal(F.entry_shape.cpu().numpy(), es)
        assert np.array_equal(F.entry_view.cpu().numpy(), ev)
        SF = O.fif_scores(q, qoff, db, w.n_views, B, off, es, ev)
        ids, sc, fl = L.gift_query_fif(V, F, Q, w.top_k, 64)
        for b in range(w.n_queries):
            assert_ranked_equal(ids.cpu().numpy()[b], sc.cpu().numpy()[b], SF[b], w.top_k)
