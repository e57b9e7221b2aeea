"""GPU parity of the second inverted file (Sec. 2.4: Eq. 7, 8, 13, 14)
against the CPU oracle."""
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth
from test_gpu_exhaustive import assert_ranked_equal

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1604_01879_amd import _lib
    return _lib


def _random_lists(rng, N, k1, crisp=False, pad=0):
    ids = np.empty((N, k1), np.int32)
    sc = np.empty((N, k1), np.float32)
    for p in range(N):
        others = rng.choice(np.delete(np.arange(N), p), size=k1 - 1, replace=False)
        ids[p] = [p] + others.tolist()
        sc[p] = [1.0] + sorted(rng.random(k1 - 1).astype(np.float32).tolist(), reverse=True)
    if crisp:
        sc[:] = 1.0
    if pad:
        ids[:pad, -1] = -1  # padding entries
    return ids, sc


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_build_sif_matches_oracle(L):
    _say("build_sif")
    rng = np.random.default_rng(0)
    N, k1 = 700, 12
    ids, sc = _random_lists(rng, N, k1, pad=30)
    sc[5, 3] = 0.0  # a zero membership has no posting
    S = L.gift_build_sif(_t(ids), _t(sc))
    torch.cuda.synchronize()
    l1, po, pid, pv = O.build_sif(ids, sc.astype(np.float64), N)
    g = S.l1.cpu().numpy().astype(np.float64)
    assert np.allclose(g[:, 0] + g[:, 1], l1, rtol=0, atol=1e-12)
    assert np.array_equal(S.post_off.cpu().numpy(), po)
    nnz = int(po[-1])
    assert np.array_equal(S.post_id.cpu().numpy()[:nnz], pid)
    assert np.array_equal(S.post_val.cpu().numpy()[:nnz].astype(np.float64), pv)


def test_rerank_golden_hand_example(L):
    _say("rerank golden")
    g = json.load(open(os.path.join(GOLD, "sif_4shape.json")))
    ids = np.array(g["nbr_ids"], np.int32)
    sc = np.array(g["nbr_scores"], np.float32)
    S = L.gift_build_sif(_t(ids), _t(sc))
    out_ids, out_s, fl = L.gift_rerank_sif(S, _t(ids), _t(sc), None, 4)
    torch.cuda.synchronize()
    out_ids, out_s = out_ids.cpu().numpy(), out_s.cpu().numpy()
    Sp = np.array(g["S_prime"])
    for p in range(4):
        ref_ids, ref_s = O.rank_topk(Sp[p][None], 4)
        assert out_ids[p].tolist() == ref_ids[0].tolist()
        assert np.allclose(out_s[p], ref_s[0], atol=1e-6)
    assert (fl.cpu().numpy() == 1).all()


@pytest.mark.parametrize("crisp", [False, True])
def test_rerank_matches_oracle(L, crisp):
    _say(f"rerank crisp={crisp}")
    rng = np.random.default_rng(3 if crisp else 4)
    N, k1, k = 400, 16, 50
    ids, sc = _random_lists(rng, N, k1, crisp=crisp)
    S = L.gift_build_sif(_t(ids), _t(sc))
    l1, po, pid, pv = O.build_sif(ids, sc.astype(np.float64), N)
    # database shapes as queries (self in the list) and outside queries
    qsel = np.arange(0, N, 37)
    q_ids = ids[qsel]
    q_sc = sc[qsel]
    oi = rng.choice(N, size=(5, k1 - 1), replace=False) if False else np.stack(
        [rng.choice(N, size=k1 - 1, replace=False) for _ in range(5)]).astype(np.int32)
    os_ = np.sort(rng.random((5, k1 - 1)).astype(np.float32), axis=1)[:, ::-1].copy()
    if crisp:
        os_[:] = 1.0
    q_ids2 = np.concatenate([oi, -np.ones((5, 1), np.int32)], axis=1)
    q_sc2 = np.concatenate([os_, np.zeros((5, 1), np.float32)], axis=1)
    all_ids = np.concatenate([q_ids, q_ids2]).astype(np.int32)
    all_sc = np.concatenate([q_sc, q_sc2]).astype(np.float32)
    self_m = np.concatenate([np.zeros(len(qsel)), np.ones(5)]).astype(np.float32)
    gi, gs, fl = L.gift_rerank_sif(S, _t(all_ids), _t(all_sc), _t(self_m), k)
    torch.cuda.synchronize()
    gi, gs = gi.cpu().numpy(), gs.cpu().numpy()
    for b in range(len(all_ids)):
        _, _, Sref = O.rerank_sif(l1, po, pid, pv, all_ids[b], all_sc[b].astype(np.float64),
                                  float(self_m[b]), k)
        assert_ranked_equal(gi[b], gs[b], Sref, k)
    # S'(x, x) = 1 for database shapes queried with their own list
    assert np.allclose(gs[:len(qsel), 0], 1.0, atol=1e-6)
    assert (gi[:len(qsel), 0] == qsel).all()


def test_sif_end_to_end_after_exhaustive(L):
    """Neighbour lists from the exhaustive path (database shapes as queries),
    S-IF built from them, out-of-database queries re-ranked with their own
    top-(k1 - 1) plus the self membership S(q, q).  The oracle runs the same
    pipeline from its own float64 scores; ranks must agree except where the
    float64 re-ranking scores are closer than the membership rounding."""
    _say("sif end to end")
    w = synth.PRESETS["c1"].scaled(n_shapes=240, dim=64, n_queries=4, m_lo=10, m_hi=64,
                                   p_dis=0.2)
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    k1, k = 10, 30
    nv = w.n_views
    # GPU
    master = _t(db)
    V = L.Views(master, nv, L.F32)
    Qdb = L.Queries(master, torch.arange(0, w.n_shapes + 1, dtype=torch.int32) * nv)
    nid, nsc, _ = L.gift_query_exhaustive(V, Qdb, k1, 64)
    Sg = L.gift_build_sif(nid, nsc)
    Q = L.Queries(_t(q), torch.from_numpy(qoff))
    qi, qs, _ = L.gift_query_exhaustive(V, Q, k1 - 1, 64)
    one = torch.ones(w.n_queries, dtype=torch.float32, device=DEV)
    gi, gs, _ = L.gift_rerank_sif(Sg, qi, qs, one, k)
    torch.cuda.synchronize()
    # oracle
    Sdb = O.exhaustive_scores(db, np.arange(w.n_shapes + 1) * nv, db, nv)
    oid, osc = O.rank_topk(Sdb, k1)
    assert np.array_equal(nid.cpu().numpy(), oid)
    l1, po, pid, pv = O.build_sif(oid, osc, w.n_shapes)
    Sq = O.exhaustive_scores(q, qoff, db, nv)
    qid_o, qsc_o = O.rank_topk(Sq, k1 - 1)
    assert np.array_equal(qi.cpu().numpy(), qid_o)
    selfs = O.self_score(q, qoff)
    gi, gs = gi.cpu().numpy(), gs.cpu().numpy()
    for b in range(w.n_queries):
        _, _, Sref = O.rerank_sif(l1, po, pid, pv, qid_o[b], qsc_o[b], selfs[b], k)
        ref_ids, ref_s = O.rank_topk(Sref[None], k)
        assert np.allclose(gs[b], ref_s[0], atol=2e-6)
        gaps = np.abs(np.diff(ref_s[0]))
        firm = np.ones(k, bool)
        firm[:-1] &= gaps > 1e-5
        firm[1:] &= gaps > 1e-5
        assert np.array_equal(gi[b][firm], ref_ids[0][firm])


def test_neighbour_augmentation_matches_oracle(L):
    """Eq. 10 on database rows (members = each shape's own top-k2, itself
    first) and on outside queries (their own list is one more member)."""
    _say("neighbour augmentation")
    rng = np.random.default_rng(21)
    N, k1, k2 = 150, 10, 4
    ids, sc = _random_lists(rng, N, k1)
    F = np.zeros((N, N))
    for p in range(N):
        F[p, ids[p]] = sc[p]
    oi, os_, nm = L.gift_augment_neighbours(_t(ids), _t(sc), _t(ids[:, :k2].copy()))
    torch.cuda.synchronize()
    ref = O.neighbour_augment(F, ids, k2)
    oi, os_ = oi.cpu().numpy(), os_.cpu().numpy()
    assert (nm.cpu().numpy() == k2).all()
    for p in range(N):
        got = np.zeros(N)
        valid = oi[p] >= 0
        got[oi[p][valid]] = os_[p][valid]
        assert list(oi[p][valid]) == sorted(oi[p][valid])
        assert np.allclose(got, ref[p], rtol=1e-6, atol=1e-7)
    # k2 = 1: unchanged rows
    oi1, os1, _ = L.gift_augment_neighbours(_t(ids), _t(sc), _t(ids[:, :1].copy()), k_out=k1)
    for p in range(0, N, 7):
        order = np.argsort(ids[p])
        assert np.array_equal(oi1.cpu().numpy()[p], ids[p][order])
        assert np.array_equal(os1.cpu().numpy()[p], sc[p][order])
    # outside queries: own list + top-(k2-1) database neighbours
    qi = np.stack([rng.choice(N, size=k1, replace=False) for _ in range(5)]).astype(np.int32)
    qv = np.sort(rng.random((5, k1)).astype(np.float32), axis=1)[:, ::-1].copy()
    mem = qi[:, :k2 - 1].copy()
    gi, gs, gn = L.gift_augment_neighbours(_t(ids), _t(sc), _t(mem), _t(qi), _t(qv))
    gi, gs = gi.cpu().numpy(), gs.cpu().numpy()
    assert (gn.cpu().numpy() == k2).all()
    # the oracle's Eq. 10 over the database rows with the queries appended as
    # rows N..N+4, each query's member list being itself then `mem`
    Fx = np.zeros((N + 5, N))
    Fx[:N] = F
    nbx = np.full((N + 5, k2), -1, np.int64)
    nbx[:N] = ids[:, :k2]
    for b in range(5):
        Fx[N + b, qi[b]] = qv[b]
        nbx[N + b] = [N + b] + mem[b].tolist()
    ref_q = O.neighbour_augment(Fx, nbx, k2)[N:]
    for b in range(5):
        got = np.zeros(N)
        valid = gi[b] >= 0
        got[gi[b][valid]] = gs[b][valid]
        assert np.allclose(got, ref_q[b], rtol=1e-6, atol=1e-7)


def test_fusion_and_co_augmentation_match_oracle(L):
    """Eq. 11 (co-augmentation through gift_augment_neighbours with the other
    measure's neighbours) followed by Eq. 9 (alpha = 0.5 and 1)."""
    _say("fusion")
    rng = np.random.default_rng(24)
    N, k1, k2 = 120, 8, 3
    i1, s1 = _random_lists(rng, N, k1)
    i2, s2 = _random_lists(rng, N, k1)
    F1 = np.zeros((N, N))
    F2 = np.zeros((N, N))
    for p in range(N):
        F1[p, i1[p]] = s1[p]
        F2[p, i2[p]] = s2[p]
    A1, A2 = O.co_augment(F1, F2, i1, i2, k2)
    a1i, a1s, _ = L.gift_augment_neighbours(_t(i1), _t(s1), _t(i2[:, :k2].copy()))
    a2i, a2s, _ = L.gift_augment_neighbours(_t(i2), _t(s2), _t(i1[:, :k2].copy()))
    for alpha in (0.5, 1.0):
        fi, fs = L.gift_fuse_activations(a1i, a1s, a2i, a2s, alpha)
        torch.cuda.synchronize()
        ref = O.fuse_activations(A1, A2, alpha)
        fi, fs = fi.cpu().numpy(), fs.cpu().numpy()
        for p in range(N):
            got = np.zeros(N)
            valid = fi[p] >= 0
            got[fi[p][valid]] = fs[p][valid]
            assert np.allclose(got, ref[p], rtol=2e-6, atol=1e-7)


def _hub_lists(rng, N, k1, hubs, n_fans, p_hub):
    """Neighbour lists where most entries point at a few hub shapes: shapes
    below n_fans list only hubs after themselves, the others take each entry
    from the hubs with probability p_hub."""
    ids = np.empty((N, k1), np.int32)
    sc = np.empty((N, k1), np.float32)
    for p in range(N):
        pool_h = hubs[hubs != p]
        if p < n_fans:
            nb = rng.choice(pool_h, size=k1 - 1, replace=False)
        else:
            nh = min(int(rng.binomial(k1 - 1, p_hub)), len(pool_h))
            nb = rng.choice(pool_h, size=nh, replace=False).tolist()
            while len(nb) < k1 - 1:
                c = int(rng.integers(0, N))
                if c != p and c not in nb:
                    nb.append(c)
            nb = np.array(nb)
        ids[p] = [p] + list(nb)
        sc[p] = [1.0] + sorted(rng.random(k1 - 1).astype(np.float32).tolist(), reverse=True)
    return ids, sc


@pytest.mark.parametrize("case", ["mixed-k100", "mixed-k1000", "fans-k1000"])
def test_rerank_hub_queries_many_passes(L, case):
    """Queries whose coordinates hold more than 4,096 postings (hub shapes
    that appear in thousands of neighbour lists) are re-ranked in several
    ranges of shape ids and still equal the oracle's Eq. 8 ranking.  "mixed":
    ordinary shapes list hubs with probability 0.6, so hub queries touch 4-8
    ranges of about 6,000 shapes.  "fans": only 700 shapes list hubs, so a hub
    query's ~6,000 postings fall on fewer shapes than k = 1,000 and the
    zero-score padding follows a multi-range result.  Flag bit 1 marks the
    queries that took more than one range."""
    _say(f"rerank hubs {case}")
    rng = np.random.default_rng(11)
    kind, _, kk = case.partition("-k")
    k = int(kk)
    hubs = np.arange(1000, 1040, dtype=np.int32)
    k1 = 20
    if kind == "mixed":
        N = 6000
        ids, sc = _hub_lists(rng, N, k1, hubs, n_fans=300, p_hub=0.6)
        plain = rng.choice(np.setdiff1d(np.arange(N), hubs), size=19, replace=False)
        q_ids = [ids[1000], ids[1017], np.concatenate([hubs[:19], [-1]]), ids[5],
                 np.concatenate([plain, [-1]])]
        q_sc = [sc[1000], sc[1017], np.concatenate([np.linspace(0.9, 0.3, 19), [0.0]]), sc[5],
                np.concatenate([np.linspace(0.8, 0.2, 19), [0.0]])]
        q_self = np.array([0, 0, 1, 0, 1], np.float32)
    else:
        N = 3000
        ids, sc = _hub_lists(rng, N, k1, hubs, n_fans=700, p_hub=0.0)
        q_ids = [np.concatenate([hubs[:19], [-1]]), ids[5], ids[2500]]
        q_sc = [np.concatenate([np.linspace(0.9, 0.3, 19), [0.0]]), sc[5], sc[2500]]
        q_self = np.array([1, 0, 0], np.float32)
    S = L.gift_build_sif(_t(ids), _t(sc))
    l1, po, pid, pv = O.build_sif(ids, sc.astype(np.float64), N)
    counts = np.diff(po)
    q_ids = np.stack(q_ids).astype(np.int32)
    q_sc = np.stack(q_sc).astype(np.float32)
    n_post = np.array([sum(int(counts[i]) for i, v in zip(r, s) if 0 <= i < N and v > 0)
                       for r, s in zip(q_ids, q_sc)])
    if kind == "mixed":
        assert n_post[:4].min() > 4 * 4096 and n_post[4] < 4096, n_post
    else:
        assert n_post[:2].min() > 4096 and n_post[2] < 4096, n_post
    gi, gs, fl = L.gift_rerank_sif(S, _t(q_ids), _t(q_sc), _t(q_self), k)
    torch.cuda.synchronize()
    gi, gs, fl = gi.cpu().numpy(), gs.cpu().numpy(), fl.cpu().numpy()
    for b in range(len(q_ids)):
        _, _, Sref = O.rerank_sif(l1, po, pid, pv, q_ids[b], q_sc[b].astype(np.float64),
                                  float(q_self[b]), k)
        if kind == "fans" and b == 0:
            assert (Sref > 0).sum() < k  # the list ends in zero-score padding
        assert_ranked_equal(gi[b], gs[b], Sref, k)
        assert fl[b] & 1
        assert bool(fl[b] & 2) == bool(n_post[b] > 4096), (b, n_post[b], fl[b])
