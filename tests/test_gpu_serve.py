"""GPU test of the continuous-batching server: results are the same when a
query runs alone and when it is batched with others under load, and equal
those of the direct calls (F-IF top-(k1-1) + self, then S-IF re-rank)."""
import sys
import time

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def test_server_alone_equals_mix():
    from paper_1604_01879_amd import _lib as L
    from paper_1604_01879_amd.serve import Server, replay_trace
    _say("server alone vs mix")
    w = synth.PRESETS["c1"].scaled(n_shapes=300, dim=128, n_queries=24, m_lo=8, m_hi=64,
                                   p_dis=0.2, seed=2)
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    master = torch.from_numpy(db).to(DEV)
    codes, scale = L.gift_quantize_views(master, L.FP8E4M3)
    V = L.Views(codes, w.n_views, L.FP8E4M3, scale, master)
    cb = master[torch.from_numpy(synth.kmeans_init_idx(db.shape[0], 32, 1))].contiguous()
    F = L.gift_build_fif(L.Views(master, w.n_views, L.F32), cb, 1)
    k1, k = 8, 20
    # S-IF from every database shape's top-k1 by Eq. 4
    Qdb = L.Queries(master, torch.arange(0, w.n_shapes + 1, dtype=torch.int32) * w.n_views)
    nid, nsc, _ = L.gift_query_fif(V, F, Qdb, k1, 32)
    S = L.gift_build_sif(nid, nsc)
    queries = [q[qoff[b]:qoff[b + 1]] for b in range(w.n_queries)]
    # direct calls
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    qi, qs, _ = L.gift_query_fif(V, F, Q, k1 - 1, 32)
    one = torch.ones(w.n_queries, dtype=torch.float32, device=DEV)
    ref_ids, ref_sc, _ = L.gift_rerank_sif(S, qi, qs, one, k)
    torch.cuda.synchronize()
    ref_ids, ref_sc = ref_ids.cpu().numpy(), ref_sc.cpu().numpy()
    srv = Server(V, F, S, top_k=k, k1=k1, rescore_r=32, max_queries=6, max_views=6 * 64,
                 max_slots=2)
    try:
        alone = []
        for v in queries:
            alone.append(srv.submit(v).result(timeout=60))
        res, lat, wall = replay_trace(srv, queries, np.zeros(len(queries)))  # all at once
        assert srv.batches < 2 * len(queries)  # the burst was batched
        for b in range(w.n_queries):
            assert np.array_equal(alone[b][0], ref_ids[b])
            assert np.array_equal(alone[b][1], ref_sc[b])
            assert np.array_equal(res[b][0], alone[b][0])
            assert np.array_equal(res[b][1], alone[b][1])
        assert (lat > 0).all()
    finally:
        srv.close()
