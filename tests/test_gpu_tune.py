"""GPU tests of the batch-plan autotuner: every candidate setting (blocks
per CU, list-tile length, narrow-tile threshold) gives the ids and exact
scores of gift_query_fif and of the oracle's Eq. 4 ranking; the tuner keeps
the fastest candidate and caches it as JSON by plan configuration."""
import json
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth
from test_gpu_exhaustive import assert_ranked_equal

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def case():
    from paper_1604_01879_amd import _lib as L
    w = synth.PRESETS["c1"].scaled(n_shapes=230, dim=128, n_queries=10, m_lo=1, m_hi=64,
                                   p_dis=0.2, seed=8)
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    cb = db[synth.kmeans_init_idx(db.shape[0], 20, 2)]
    master = torch.from_numpy(db).to(DEV)
    F = L.gift_build_fif(L.Views(master, w.n_views, L.F32), torch.from_numpy(cb).to(DEV), 2)
    S = O.fif_scores(q, qoff, db, w.n_views, cb, *O.build_fif(O.assign(db, cb, 2), 20,
                                                                w.n_views))
    return L, w, db, q, qoff, master, F, S


@pytest.mark.parametrize("dtype_name", ["f32", "bf16", "fp8"])
def test_every_candidate_gives_the_same_ranking(case, dtype_name):
    from paper_1604_01879_amd.tune import CANDIDATES
    L, w, db, q, qoff, master, F, S = case
    _say(f"tuning candidates {dtype_name}")
    dt = {"f32": L.F32, "bf16": L.BF16, "fp8": L.FP8E4M3}[dtype_name]
    if dt == L.F32:
        V = L.Views(master, w.n_views, L.F32)
    else:
        codes, scale = L.gift_quantize_views(master, dt)
        V = L.Views(codes, w.n_views, dt, scale, master)
    k, R = 12, w.n_shapes  # every shape rescored: the exact top k whatever the first pass
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    ref_ids, ref_sc, _ = L.gift_query_fif(V, F, Q, k, R)
    ref_ids, ref_sc = ref_ids.cpu().numpy(), ref_sc.cpu().numpy()
    n_q, n_v = len(qoff) - 1, int(qoff[-1])
    for cand in CANDIDATES:
        plan = L.FifPlan(V, F, 12, 12 * 64, 64, k, R, **cand)
        plan.views[:n_v] = torch.from_numpy(q).to(DEV)
        plan.offsets[:n_q + 1] = torch.from_numpy(qoff).to(DEV)
        torch.cuda.synchronize()
        plan.run(n_q, n_v)
        plan.stream.synchronize()
        assert plan.error() == 0, cand
        ids, sc = plan.ids[:n_q].cpu().numpy(), plan.scores[:n_q].cpu().numpy()
        assert np.array_equal(ids, ref_ids), cand
        assert np.array_equal(sc, ref_sc), cand
        for b in range(n_q):
            assert_ranked_equal(ids[b], sc[b], S[b], k)
        plan.close()


def test_tuner_keeps_the_fastest_and_caches_it(case, tmp_path, monkeypatch):
    from paper_1604_01879_amd import tune
    L, w, db, q, qoff, master, F, S = case
    _say("tuner and cache")
    V = L.Views(master, w.n_views, L.F32)
    cands = tune.CANDIDATES[:4]
    path = str(tmp_path / "tuning.json")
    qv = torch.from_numpy(q).to(DEV)
    best, entry = tune.tune_plan(V, F, qv, qoff, 64, 10, 40, candidates=cands, reps=2,
                                 cache_path=path)
    assert best in [dict(c) for c in cands]
    assert len(entry["ms_grid"]) == 4 and all(g["ms"] > 0 for g in entry["ms_grid"])
    assert min(entry["ms_grid"], key=lambda g: g["ms"])["ms"] == \
        next(g["ms"] for g in entry["ms_grid"] if all(g[k] == best[k] for k in best))
    stored = json.load(open(path))
    key = tune.config_key(V, F, len(qoff) - 1, int(qoff[-1]), 64, 10, 40)
    assert stored[key]["best"] == best
    # a second call reads the cache and times nothing
    monkeypatch.setattr(tune, "time_plan", lambda *a, **k: pytest.fail("timed again"))
    best2, _ = tune.tune_plan(V, F, qv, qoff, 64, 10, 40, candidates=cands, cache_path=path)
    assert best2 == best
