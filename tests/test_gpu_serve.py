"""GPU tests of the continuous-batching server: each result is the same when
a query runs alone and when it is batched with others under load, equals the
direct calls (F-IF top-(k1-1) + self, then the S-IF re-rank) and the oracle
pipeline (Eq. 4 lists, Eq. 7 S-IF, Eq. 8 re-ranking); and a memory budget
that holds a single small slot makes queries wait and split into batches
that fit it, with the same results."""
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
def setup():
    """300 shapes in e4m3 storage, a 32-word F-IF (MA 1), and the S-IF of
    every shape's top-k1 by Eq. 4 (every shape rescored, so each list is the
    exact Eq. 4 top-k1)."""
    from paper_1604_01879_amd import _lib as L
    w = synth.PRESETS["c1"].scaled(n_shapes=300, dim=128, n_queries=24, m_lo=8, m_hi=64,
                                   p_dis=0.2, seed=2)
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    master = torch.from_numpy(db).to(DEV)
    codes, scale = L.gift_quantize_views(master, L.FP8E4M3)
    V = L.Views(codes, w.n_views, L.FP8E4M3, scale, master)
    cb_np = db[synth.kmeans_init_idx(db.shape[0], 32, 1)]
    F = L.gift_build_fif(L.Views(master, w.n_views, L.F32), torch.from_numpy(cb_np).to(DEV), 1)
    k1, k, R = 8, 20, w.n_shapes
    Qdb = L.Queries(master, torch.arange(0, w.n_shapes + 1, dtype=torch.int32) * w.n_views)
    nid, nsc, _ = L.gift_query_fif(V, F, Qdb, k1, R)
    S = L.gift_build_sif(nid, nsc)
    torch.cuda.synchronize()
    return L, w, db, q, qoff, cb_np, V, F, S, k1, k, R


def _oracle_pipeline(w, db, q, qoff, cb, k1, k):
    """Eq. 4 top-k1 of every database shape (S-IF, Eq. 7) and top-(k1 - 1) of
    every query plus itself, re-ranked by Eq. 8; memberships rounded to
    float32 as the library returns scores."""
    off, es, ev = O.build_fif(O.assign(db, cb, 1), len(cb), w.n_views)
    N = w.n_shapes
    Sdb = O.fif_scores(db, np.arange(N + 1) * w.n_views, db, w.n_views, cb, off, es, ev)
    ids, sc = O.rank_topk(Sdb, k1)
    l1, po, pid, pv = O.build_sif(ids, sc.astype(np.float32).astype(np.float64), N)
    Sq = O.fif_scores(q, qoff, db, w.n_views, cb, off, es, ev)
    qi, qv = O.rank_topk(Sq, k1 - 1)
    out = []
    for b in range(len(qoff) - 1):
        _, _, Sfull = O.rerank_sif(l1, po, pid, pv, qi[b],
                                   qv[b].astype(np.float32).astype(np.float64), 1.0, k)
        out.append(Sfull)
    return out


def _assert_like_oracle(ids, sc, Sref, k, tie=1e-6):
    ref_ids, ref_s = O.rank_topk(Sref[None], k)
    ref_ids, ref_s = ref_ids[0], ref_s[0]
    assert len(set(ids.tolist())) == k
    assert np.allclose(sc, Sref[ids], rtol=REL, atol=1e-7)
    assert np.all(np.abs(Sref[ids] - ref_s) <= tie)
    gaps = np.abs(np.diff(ref_s))
    near = np.zeros(k, bool)
    near[:-1] |= gaps <= tie
    near[1:] |= gaps <= tie
    assert np.array_equal(ids[~near], ref_ids[~near])


def _direct(L, w, q, qoff, V, F, S, k1, k, R):
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    qi, qs, _ = L.gift_query_fif(V, F, Q, k1 - 1, R)
    one = torch.ones(w.n_queries, dtype=torch.float32, device=DEV)
    ref_ids, ref_sc, _ = L.gift_rerank_sif(S, qi, qs, one, k)
    torch.cuda.synchronize()
    return ref_ids.cpu().numpy(), ref_sc.cpu().numpy()


def test_server_alone_equals_mix_and_oracle(setup):
    from paper_1604_01879_amd.serve import Server, replay_trace
    L, w, db, q, qoff, cb, V, F, S, k1, k, R = setup
    _say("server alone vs mix vs oracle")
    ref_ids, ref_sc = _direct(L, w, q, qoff, V, F, S, k1, k, R)
    Sref = _oracle_pipeline(w, db, q, qoff, cb, k1, k)
    queries = [q[qoff[b]:qoff[b + 1]] for b in range(w.n_queries)]
    srv = Server(V, F, S, top_k=k, k1=k1, rescore_r=R, max_queries=6, max_m=64, max_slots=2)
    try:
        alone = [srv.submit(v).result(timeout=60) for v in queries]
        res, lat, wall = replay_trace(srv, queries, np.zeros(len(queries)))  # all at once
        assert srv.stats["batches"] < 2 * len(queries)  # the burst was batched
        for b in range(w.n_queries):
            assert np.array_equal(alone[b][0], ref_ids[b])
            assert np.array_equal(alone[b][1], ref_sc[b])
            assert np.array_equal(res[b][0], alone[b][0])
            assert np.array_equal(res[b][1], alone[b][1])
            _assert_like_oracle(res[b][0], res[b][1], Sref[b], k)
        assert (lat > 0).all()
    finally:
        srv.close()


def test_server_memory_budget_makes_queries_wait(setup):
    """A budget that holds one slot of the 4-query class (and nothing larger)
    serves a burst of 24 queries of up to 64 views: the server creates that
    one slot, queries wait for it (memory waits), batches hold at most 4
    queries, and every result is the one the query gets alone."""
    from paper_1604_01879_amd.serve import Server, replay_trace
    L, w, db, q, qoff, cb, V, F, S, k1, k, R = setup
    _say("server under a one-slot memory budget")
    ref_ids, ref_sc = _direct(L, w, q, qoff, V, F, S, k1, k, R)
    queries = [q[qoff[b]:qoff[b + 1]] for b in range(w.n_queries)]
    probe = Server(V, F, S, top_k=k, k1=k1, rescore_r=R, max_queries=16, max_m=64, max_slots=1,
                   prewarm=False)
    classes, sizes = probe.classes, probe.slot_bytes
    probe.close()
    i4 = classes.index((4, 256))
    budget = sizes[i4] + 256
    assert budget < sizes[i4 + 1]  # no room for the 16-query class
    srv = Server(V, F, S, top_k=k, k1=k1, rescore_r=R, max_queries=16, max_m=64, max_slots=3,
                 mem_budget_bytes=budget)
    try:
        assert len(srv.slots) == 1 and srv.slots[0].q_cap == 4
        res, lat, wall = replay_trace(srv, queries, np.zeros(len(queries)))
        st = srv.stats
        assert st["memory_waits"] > 0
        assert st["batches"] >= len(queries) // 4
        assert st["max_busy_slots"] == 1 and st["peak_bytes"] <= budget
        for b in range(w.n_queries):
            assert np.array_equal(res[b][0], ref_ids[b])
            assert np.array_equal(res[b][1], ref_sc[b])
    finally:
        srv.close()


def test_copy_async_round_trip():
    """gift_copy_async moves bytes host -> device -> host on a stream, in
    the order queued, for pinned host and device tensors."""
    from paper_1604_01879_amd import _lib as L
    print("[gpu] copy_async round trip", flush=True)
    st = torch.cuda.Stream()
    src = torch.arange(1 << 16, dtype=torch.int32).pin_memory()
    dev = torch.empty(1 << 16, dtype=torch.int32, device="cuda:0")
    back = torch.zeros(1 << 16, dtype=torch.int32).pin_memory()
    L.copy_async(dev, src, st)
    L.copy_async(back, dev, st)
    st.synchronize()
    assert torch.equal(back, src)
    with pytest.raises(ValueError):
        L.copy_async(back[:10], dev, st)


def test_plan_serve_equals_separate_calls(setup):
    """gift_fif_plan_serve (copies in, plan, optional S-IF re-rank, copies
    out, one call) returns what the separate calls return, bit for bit: two
    batches in a row, the second smaller, without and with the re-rank."""
    L, w, db, q, qoff, cb, V, F, S, k1, k, R = setup
    GiftError = L.GiftError
    _say("plan serve vs separate calls")
    kp = k1 - 1
    plan = L.FifPlan(V, F, 6, 6 * 64, 64, kp, R)
    st = plan.stream
    hv = torch.zeros((6 * 64, w.dim), dtype=torch.float32).pin_memory()
    ho = torch.zeros(7, dtype=torch.int32).pin_memory()
    hid = torch.zeros((6, k), dtype=torch.int32).pin_memory()
    hsc = torch.zeros((6, k), dtype=torch.float32).pin_memory()
    hfl = torch.zeros(6, dtype=torch.int32).pin_memory()
    one = torch.ones(6, dtype=torch.float32, device=DEV)
    rr_ids = torch.zeros((6, k), dtype=torch.int32, device=DEV)
    rr_sc = torch.zeros((6, k), dtype=torch.float32, device=DEV)
    rr_fl = torch.zeros(6, dtype=torch.int32, device=DEV)
    head = (plan.handle, hv.data_ptr(), ho.data_ptr())
    no_rr = (0, None, None, None, None, None, 0, None, None, None)
    rr = (S.n_shapes, S.l1.data_ptr(), S.post_off.data_ptr(), S.post_id.data_ptr(),
          S.post_val.data_ptr(), one.data_ptr(), k, rr_ids.data_ptr(), rr_sc.data_ptr(),
          rr_fl.data_ptr())
    for b0, b1 in ((0, 5), (5, 7)):
        n = b1 - b0
        v0, v1 = int(qoff[b0]), int(qoff[b1])
        nv = v1 - v0
        hv[:nv] = torch.from_numpy(q[v0:v1])
        ho[:n + 1] = torch.from_numpy((qoff[b0:b1 + 1] - v0).astype(np.int32))
        # without the re-rank: the plan's own top-kp, scores and flags
        L.fif_plan_serve(*head, n, nv, *no_rr, hid.data_ptr(), hsc.data_ptr(), hfl.data_ptr(),
                         st.cuda_stream)
        st.synchronize()
        got = (hid.view(-1)[:n * kp].clone(), hsc.view(-1)[:n * kp].clone(), hfl[:n].clone())
        plan.views[:nv].copy_(hv[:nv].to(DEV))
        plan.offsets[:n + 1].copy_(ho[:n + 1].to(DEV))
        torch.cuda.synchronize()
        plan.run(n, nv)
        st.synchronize()
        assert torch.equal(got[0], plan.ids[:n].reshape(-1).cpu())
        assert torch.equal(got[1], plan.scores[:n].reshape(-1).cpu())
        assert torch.equal(got[2], plan.flags[:n].cpu())
        ref_ids, ref_sc, ref_fl = L.gift_rerank_sif(S, plan.ids[:n], plan.scores[:n], one[:n], k)
        torch.cuda.synchronize()
        # with the re-rank
        L.fif_plan_serve(*head, n, nv, *rr, hid.data_ptr(), hsc.data_ptr(), hfl.data_ptr(),
                         st.cuda_stream)
        st.synchronize()
        assert torch.equal(hid[:n], ref_ids.cpu())
        assert torch.equal(hsc[:n], ref_sc.cpu())
        assert torch.equal(hfl[:n], ref_fl.cpu())
    # host-side argument checks (nothing is queued)
    with pytest.raises(GiftError) as e:
        L.fif_plan_serve(*head, 7, 64, *no_rr, hid.data_ptr(), hsc.data_ptr(), hfl.data_ptr(),
                         st.cuda_stream)
    assert e.value.status == L.ECAPACITY
    bad = rr[:7] + (None,) + rr[8:]
    with pytest.raises(GiftError) as e:
        L.fif_plan_serve(*head, 1, 8, *bad, hid.data_ptr(), hsc.data_ptr(), hfl.data_ptr(),
                         st.cuda_stream)
    assert e.value.status == L.EINVAL
