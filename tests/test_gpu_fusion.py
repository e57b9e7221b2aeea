"""GPU parity of the two-measure search (Sec. 2.4: Eq. 7 activations, Eq. 11
co-augmentation, Eq. 9 fusion with alpha = 0.5, Eq. 8 through the S-IF)
against the same chain run by the CPU oracle: exhaustive Eq. 3 neighbour
lists of the database and of the queries under each measure, dense
co-augmentation and fusion, the oracle's S-IF and its Eq. 8 re-ranking."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
REL = 1e-5


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1604_01879_amd import _lib
    return _lib


def oracle_two_measure(dbs, qs, qoff, nv, k1, k2, alpha, top_k):
    """The fused re-ranking by the oracle: per measure the exact top-k1 of
    every database shape and the top-(k1 - 1) of every query by Eq. 3 (their
    memberships rounded to float32, as the library returns scores), dense
    activations with the queries appended as rows N..N+B-1, Eq. 11 with each
    query's member list = itself then its top-(k2 - 1) database neighbours,
    Eq. 9, the S-IF of the fused database rows and Eq. 8 with the query's
    fused self membership."""
    N = dbs[0].shape[0] // nv
    B = len(qoff) - 1
    F, nbr = [], []
    for db, q in zip(dbs, qs):
        S = O.exhaustive_scores(db, np.arange(N + 1) * nv, db, nv)
        ids, sc = O.rank_topk(S, k1)
        Sq = O.exhaustive_scores(q, qoff, db, nv)
        qi, qv = O.rank_topk(Sq, k1 - 1)
        sc = sc.astype(np.float32).astype(np.float64)
        qv = qv.astype(np.float32).astype(np.float64)
        D = np.zeros((N + B, N))
        for p in range(N):
            D[p, ids[p]] = sc[p]
        for b in range(B):
            D[N + b, qi[b]] = qv[b]
        nb = np.full((N + B, k2), -1, np.int64)
        nb[:N] = ids[:, :k2]
        nb[N:, 0] = N + np.arange(B)
        nb[N:, 1:] = qi[:, :k2 - 1]
        F.append(D)
        nbr.append(nb)
    A1, A2 = O.co_augment(F[0], F[1], nbr[0], nbr[1], k2)
    Ff = O.fuse_activations(A1, A2, alpha)
    width = max(int((Ff[:N] > 0).sum(axis=1).max()), 1)
    db_ids = np.full((N, width), -1, np.int64)
    db_sc = np.zeros((N, width))
    for p in range(N):
        nz = np.flatnonzero(Ff[p] > 0)
        db_ids[p, :len(nz)] = nz
        db_sc[p, :len(nz)] = Ff[p, nz]
    l1, po, pid, pv = O.build_sif(db_ids, db_sc, N)
    # the query's own membership 1 is averaged over its k2 members under
    # each measure, then fused like every coordinate
    q_self = float(O.fuse_activations(np.array([1.0 / k2]), np.array([1.0 / k2]), alpha)[0])
    out = []
    for b in range(B):
        nz = np.flatnonzero(Ff[N + b] > 0)
        _, _, Sfull = O.rerank_sif(l1, po, pid, pv, nz, Ff[N + b, nz], q_self, top_k)
        out.append(Sfull)
    return out


def _assert_ranked_close(ids, scores, S, k, tie=2e-5):
    """The GPU list against the oracle's float64 Eq. 8 row: distinct ids, each
    score within REL of the oracle's score of that id, every rank's oracle
    score equal to the oracle's rank-r score up to `tie` (the fused rows are
    float32 on the GPU), and ids equal wherever the oracle's neighbouring
    scores differ by more than `tie`."""
    ref_ids, ref_s = O.rank_topk(S[None], k)
    ref_ids, ref_s = ref_ids[0], ref_s[0]
    assert len(set(ids.tolist())) == k
    assert np.allclose(scores, S[ids], rtol=REL, atol=1e-7)
    assert np.all(np.abs(S[ids] - ref_s) <= tie)
    gaps = np.abs(np.diff(ref_s))
    near = np.zeros(k, bool)
    near[:-1] |= gaps <= tie
    near[1:] |= gaps <= tie
    assert np.array_equal(ids[~near], ref_ids[~near])


@pytest.mark.parametrize("k2", [1, 4])
def test_two_measure_search_matches_oracle_chain(L, k2):
    from paper_1604_01879_amd.fusion import TwoMeasureIndex
    _say(f"two-measure search k2={k2}")
    w = synth.PRESETS["c1"].scaled(n_shapes=200, dim=128, n_queries=6, m_lo=16, m_hi=64,
                                   p_dis=0.2, seed=5)
    db1, _, _ = synth.make_db(w)
    q1, qoff, _ = synth.make_queries(w)
    db2, q2, qoff2 = synth.make_second_measure(w, dim=96)
    assert np.array_equal(qoff, qoff2)
    k1, alpha, top_k = 10, 0.5, 20
    V1 = L.Views(torch.from_numpy(db1).to(DEV), w.n_views, L.F32)
    V2 = L.Views(torch.from_numpy(db2).to(DEV), w.n_views, L.F32)
    idx = TwoMeasureIndex(V1, V2, k1=k1, k2=k2, alpha=alpha, chunk=64)
    Q1 = L.Queries(torch.from_numpy(q1).to(DEV), torch.from_numpy(qoff))
    Q2 = L.Queries(torch.from_numpy(q2).to(DEV), torch.from_numpy(qoff))
    ids, sc = idx.query(Q1, Q2, top_k)
    torch.cuda.synchronize()
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    ref = oracle_two_measure((db1, db2), (q1, q2), qoff, w.n_views, k1, k2, alpha, top_k)
    for b in range(len(qoff) - 1):
        assert (ref[b] > 0).sum() >= top_k  # the list is no zero-score padding
        _assert_ranked_close(ids[b], sc[b], ref[b], top_k)
