"""gift_query_exhaustive_static (the exhaustive query on the library's static
device scratch, for callers that cannot allocate) against
gift_query_exhaustive on a caller workspace and against the oracle's Eq. 3
ranking: two calls in a row, the second with a smaller batch, so the second
runs on scratch that still holds the first call's contents."""
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
def L():
    from paper_1604_01879_amd import _lib
    return _lib


def _case(L, dtype, n_shapes, dim, n_queries, m, seed):
    w = synth.PRESETS["c1"].scaled(n_shapes=n_shapes, dim=dim, n_queries=n_queries, m_lo=m[0],
                                   m_hi=m[1], p_dis=0.2, seed=seed)
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    master = torch.from_numpy(db).to(DEV)
    if dtype == L.F32:
        V = L.Views(master, w.n_views, L.F32)
    else:
        codes, scale = L.gift_quantize_views(master, dtype)
        V = L.Views(codes, w.n_views, dtype, scale, master)
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff),
                  offsets_host=torch.from_numpy(qoff))
    return w, db, q, qoff, V, Q


@pytest.mark.parametrize("dtype_name", ["f32", "fp8"])
def test_static_scratch_equals_workspace_call(L, dtype_name):
    dt = {"f32": L.F32, "fp8": L.FP8E4M3}[dtype_name]
    # the first batch is the larger one; the second reuses the scratch
    for n_shapes, dim, B, m, k, R, seed in ((700, 256, 7, (1, 64), 12, 40, 3),
                                            (300, 128, 3, (5, 20), 5, 16, 4)):
        _say(f"static scratch {dtype_name}: {n_shapes} shapes x {dim}, {B} queries, seed {seed}")
        w, db, q, qoff, V, Q = _case(L, dt, n_shapes, dim, B, m, seed)
        need = L.query_exhaustive_static_bytes(V, Q, k, R)
        assert 0 < need <= L.STATIC_SCRATCH_BYTES
        ids, sc, fl = L.gift_query_exhaustive_static(V, Q, k, R)
        torch.cuda.synchronize()
        ref_ids, ref_sc, ref_fl = L.gift_query_exhaustive(V, Q, k, R)
        torch.cuda.synchronize()
        # same kernels on the same inputs: bit-identical outputs
        assert torch.equal(ids, ref_ids)
        assert torch.equal(sc, ref_sc)
        assert torch.equal(fl, ref_fl)
        # and the oracle's exact Eq. 3 ranking
        S = O.exhaustive_scores(q, qoff, db, w.n_views)
        ids_h, sc_h, fl_h = ids.cpu().numpy(), sc.cpu().numpy(), fl.cpu().numpy()
        for b in range(B):
            assert_ranked_equal(ids_h[b], sc_h[b], S[b], k)
        if dt == L.F32:
            assert fl_h.all()

