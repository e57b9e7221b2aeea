"""GPU tests of the batch plan: the F-IF path as one persistent kernel plus
ranking kernels captured in a HIP graph.  Its results must equal those of
gift_query_fif on the same batch (and so the oracle's), for every replay."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth
from test_gpu_exhaustive import assert_ranked_equal, assert_returned_exact

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1604_01879_amd import _lib
    return _lib


def _setup(L, dtype, n_shapes=260, dim=128, K=24, ma=2, B=9, seed=0):
    if dtype in (L.MXFP8, L.MXFP4):
        dim = 256  # MX storage needs whole 128 / 256-value K-tiles
    w = synth.PRESETS["c1"].scaled(n_shapes=n_shapes, dim=dim, n_queries=B, m_lo=1, m_hi=64,
                                   p_dis=0.2, seed=seed)
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    cb = db[synth.kmeans_init_idx(db.shape[0], K, 3)]
    master = torch.from_numpy(db).to(DEV)
    V32 = L.Views(master, w.n_views, L.F32)
    F = L.gift_build_fif(V32, torch.from_numpy(cb).to(DEV), ma)
    if dtype == L.F32:
        V = V32
    else:
        codes, scale = L.gift_quantize_views(master, dtype)
        V = L.Views(codes, w.n_views, dtype, scale, master)
    return w, db, q, qoff, cb, V, F


def _load(plan, q, qoff):
    n_q = len(qoff) - 1
    plan.views[:qoff[-1]] = torch.from_numpy(q).to(DEV)
    plan.offsets[:n_q + 1] = torch.from_numpy(qoff).to(DEV)
    torch.cuda.synchronize()  # the plan runs on its own stream
    return n_q, int(qoff[-1])


# "bf16_263": a shape count that is not a multiple of 4 (the per-query mean
# then reads one shape per load instead of four).  gemm 1: the codeword dots
# as items of the persistent kernel; 2: a separate GEMM kernel before it.
@pytest.mark.parametrize("gemm", [1, 2])
@pytest.mark.parametrize("dtype_name", ["f32", "bf16", "fp8", "mxfp8", "mxfp4", "bf16_263"])
def test_plan_equals_query_fif(L, dtype_name, gemm):
    _say(f"plan vs query_fif {dtype_name} gemm {gemm}")
    name, _, ns = dtype_name.partition("_")
    dt = {"f32": L.F32, "bf16": L.BF16, "fp8": L.FP8E4M3, "mxfp8": L.MXFP8,
          "mxfp4": L.MXFP4}[name]
    w, db, q, qoff, cb, V, F = _setup(L, dt, n_shapes=int(ns) if ns else 260)
    torch.cuda.synchronize()
    _say("index built")
    k, R = 15, 60
    plan = L.FifPlan(V, F, max_queries=12, max_views=12 * 64, max_views_per_query=64, top_k=k,
                     rescore_r=R, gemm=gemm)
    _say("plan created")
    S = O.fif_scores(q, qoff, db, w.n_views, cb, *O.build_fif(O.assign(db, cb, 2), 24,
                                                                w.n_views))
    # full batch, then a smaller one (fewer queries and views) on the same plan
    for sub in (len(qoff) - 1, 4):
        qo = qoff[:sub + 1]
        qq = q[:qo[-1]]
        Q = L.Queries(torch.from_numpy(qq).to(DEV), torch.from_numpy(qo))
        ref_ids, ref_sc, ref_fl = L.gift_query_fif(V, F, Q, k, R)
        ref_s1, _ = L.gift_score_fif(V, F, Q)
        torch.cuda.synchronize()
        _say(f"query_fif {sub} queries done")
        n_q, n_v = _load(plan, qq, qo)
        for eager in (False, True, False, True):
            plan.run(n_q, n_v, eager=eager)
            plan.stream.synchronize()
            _say(f"plan run eager={eager} done")
            assert plan.error() == 0
            # the first pass is gift_score_fif's, bit for bit (same tiles,
            # products and order), on every run
            s1 = plan.first_pass(n_q)
            plan.stream.synchronize()
            assert torch.equal(s1, ref_s1), int((s1 != ref_s1).sum())
            ids = plan.ids[:n_q].cpu().numpy()
            sc = plan.scores[:n_q].cpu().numpy()
            assert np.array_equal(ids, ref_ids.cpu().numpy())
            assert np.array_equal(sc, ref_sc.cpu().numpy())
            fl = plan.flags[:n_q].cpu().numpy()
            # same first pass and the same per-query bound: the same flags;
            # a set flag must be sound (the ids are the exact top k)
            assert np.array_equal(fl, ref_fl.cpu().numpy())
            for b in range(n_q):
                if fl[b] & 1:
                    assert_ranked_equal(ids[b], sc[b], S[b], k)
            for b in range(n_q):
                if dt in (L.MXFP8, L.MXFP4):
                    # MX first passes are never certified complete: check that
                    # each returned score is the exact Eq. 4 score of its id,
                    # in (score desc, id asc) order
                    assert np.allclose(sc[b], S[b][ids[b]], rtol=1e-5, atol=1e-6)
                    assert all((sc[b][t], -ids[b][t]) >= (sc[b][t + 1], -ids[b][t + 1])
                               for t in range(k - 1))
                else:
                    assert_ranked_equal(ids[b], sc[b], S[b], k)
    plan.close()


def test_plan_replays_with_eager_work_between(L):
    _say("plan replays")
    w, db, q, qoff, cb, V, F = _setup(L, L.F32, seed=4)
    k, R = 10, 40
    plan = L.FifPlan(V, F, max_queries=9, max_views=9 * 64, max_views_per_query=64, top_k=k,
                     rescore_r=R)
    n_q, n_v = _load(plan, q, qoff)
    plan.run(n_q, n_v)
    plan.stream.synchronize()
    first = (plan.ids.clone(), plan.scores.clone())
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    for _ in range(4):
        L.gift_query_fif(V, F, Q, k, R)  # eager work on another stream in between
        torch.cuda.synchronize()
        plan.run(n_q, n_v)
        plan.stream.synchronize()
        assert torch.equal(plan.ids, first[0])
        assert torch.equal(plan.scores, first[1])
    ph = plan.phase_us()
    assert len(ph) == 9 and all(t >= 0 for t in ph) and ph[7] > 0  # the list scan ran
    # phase end times: every phase ran, and a phase that waits for others
    # ends after them (split/quantize 0, dots 1, select 3, offsets 4,
    # grouping 5, active tiles 6, scan 7, mean 8; the clear, 2, has no items
    # of its own: the dot-tile items clear the match buffer)
    end = plan.phase_end_us()
    assert len(end) == 9 and end[2] == 0 and all(t > 0 for i, t in enumerate(end) if i != 2), end
    for later, earlier in ((1, 0), (3, 1), (4, 3), (5, 4), (6, 5), (7, 6), (8, 7)):
        assert end[later] >= end[earlier], (later, earlier, end)
    assert end[8] < 1e6  # microseconds of one small batch
    plan.close()


def test_plan_alone_and_in_the_mix(L):
    """A query's result is identical when it runs alone and when it shares
    the batch with others."""
    _say("plan alone vs mix")
    w, db, q, qoff, cb, V, F = _setup(L, L.BF16, seed=6, B=8)
    k, R = 12, 48
    plan = L.FifPlan(V, F, max_queries=8, max_views=8 * 64, max_views_per_query=64, top_k=k,
                     rescore_r=R)
    n_q, n_v = _load(plan, q, qoff)
    plan.run(n_q, n_v)
    plan.stream.synchronize()
    mix_ids, mix_sc = plan.ids[:n_q].cpu().numpy(), plan.scores[:n_q].cpu().numpy()
    mix_fl = plan.flags[:n_q].cpu().numpy()
    for b in (0, 5, 7):
        lo, hi = qoff[b], qoff[b + 1]
        _load(plan, q[lo:hi], np.array([0, hi - lo], np.int32))
        plan.run(1, int(hi - lo))
        plan.stream.synchronize()
        assert np.array_equal(plan.ids[0].cpu().numpy(), mix_ids[b])
        assert np.array_equal(plan.scores[0].cpu().numpy(), mix_sc[b])
        # the certificate uses the query's own view count, not the batch's
        assert int(plan.flags[0].item()) == int(mix_fl[b])
    plan.close()


def test_plan_rejects_oversized_batch(L):
    _say("plan capacity")
    w, db, q, qoff, cb, V, F = _setup(L, L.F32, B=3)
    plan = L.FifPlan(V, F, max_queries=3, max_views=100, max_views_per_query=64, top_k=5,
                     rescore_r=20)
    with pytest.raises(L.GiftError) as e:
        plan.run(4, 50)
    assert e.value.status == L.ECAPACITY
    with pytest.raises(L.GiftError):
        plan.run(2, 101)
    plan.close()


@pytest.mark.parametrize("gemm", [1, 2])
def test_plan_large_batch_equals_query_fif(L, gemm):
    """A batch of more than 512 query views: the word selection takes one
    wave per view instead of a whole block, and the per-query mean spans
    several 4,096-shape items; first pass, ids and scores still equal
    gift_query_fif's and the ids the oracle's."""
    _say(f"plan large batch gemm {gemm}")
    w, db, q, qoff, cb, V, F = _setup(L, L.BF16, n_shapes=4500, B=24, seed=9)
    assert qoff[-1] > 512, "the batch must exceed the per-view selection limit"
    k, R = 10, 40
    plan = L.FifPlan(V, F, max_queries=24, max_views=24 * 64, max_views_per_query=64, top_k=k,
                     rescore_r=R, gemm=gemm)
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    ref_ids, ref_sc, _ = L.gift_query_fif(V, F, Q, k, R)
    ref_s1, _ = L.gift_score_fif(V, F, Q)
    torch.cuda.synchronize()
    n_q, n_v = _load(plan, q, qoff)
    for _ in range(2):
        plan.run(n_q, n_v)
        plan.stream.synchronize()
        assert plan.error() == 0
        s1 = plan.first_pass(n_q)
        plan.stream.synchronize()
        assert torch.equal(s1, ref_s1), int((s1 != ref_s1).sum())
        assert np.array_equal(plan.ids[:n_q].cpu().numpy(), ref_ids.cpu().numpy())
        assert np.array_equal(plan.scores[:n_q].cpu().numpy(), ref_sc.cpu().numpy())
    S = O.fif_scores(q, qoff, db, w.n_views, cb, *O.build_fif(O.assign(db, cb, 2), 24, w.n_views))
    ids, sc, fl = (t[:n_q].cpu().numpy() for t in (plan.ids, plan.scores, plan.flags))
    for b in range(n_q):
        if fl[b] & 1:
            assert_ranked_equal(ids[b], sc[b], S[b], k)
    plan.close()


@pytest.mark.parametrize("dtype_name", ["f32", "fp8"])
def test_small_plan_split_rescore_equals_query_fif(L, dtype_name):
    """A plan of at most 4 queries of up to 64 views splits the approximate
    rescore phase over K (4 blocks per work item, partial tiles added in
    split order): ids, scores and flags still equal gift_query_fif's (one
    block per item over the whole K range), and the ids the oracle's."""
    _say(f"small plan split rescore {dtype_name}")
    dt = {"f32": L.F32, "fp8": L.FP8E4M3}[dtype_name]
    w, db, q, qoff, cb, V, F = _setup(L, dt, n_shapes=300, dim=512, B=4, seed=11)
    k, R = 10, 40
    plan = L.FifPlan(V, F, max_queries=4, max_views=4 * 64, max_views_per_query=64, top_k=k,
                     rescore_r=R)
    S = O.fif_scores(q, qoff, db, w.n_views, cb, *O.build_fif(O.assign(db, cb, 2), 24,
                                                                w.n_views))
    for sub in (4, 1):
        qo = qoff[:sub + 1]
        qq = q[:qo[-1]]
        Q = L.Queries(torch.from_numpy(qq).to(DEV), torch.from_numpy(qo))
        ref_ids, ref_sc, ref_fl = L.gift_query_fif(V, F, Q, k, R)
        torch.cuda.synchronize()
        n_q, n_v = _load(plan, qq, qo)
        for _ in range(2):
            plan.run(n_q, n_v)
            plan.stream.synchronize()
            assert plan.error() == 0
            ids, sc = plan.ids[:n_q].cpu().numpy(), plan.scores[:n_q].cpu().numpy()
            assert np.array_equal(ids, ref_ids.cpu().numpy())
            assert np.array_equal(sc, ref_sc.cpu().numpy())
            assert np.array_equal(plan.flags[:n_q].cpu().numpy(), ref_fl.cpu().numpy())
        fl = plan.flags[:n_q].cpu().numpy()
        for b in range(n_q):
            assert_returned_exact(ids[b], sc[b], S[b], k)
            if dt == L.F32 or fl[b] & 1:
                assert_ranked_equal(ids[b], sc[b], S[b], k)
    plan.close()
