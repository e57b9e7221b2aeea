"""GPU parity at the feature width and vocabulary size of the 12,000-shape
workloads (d = 4096, K = 4096), on a database reduced to 256 shapes so the
float64 oracle finishes in seconds: quantizer words at MA 1 and 3, the
F-IF lists, and the ranked ids of Eq. 3 and Eq. 4 in float32 and e4m3
storage.  The d = 4096 rows run the full 32-sub-tile K loops of the score,
scan, quantizer and rescore kernels; K = 4096 runs the quantizer's many
codeword tiles and a mostly empty, many-list index."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import synth
from test_gpu_exhaustive import assert_flags_as_predicted, assert_ranked_equal, assert_returned_exact
from test_gpu_fif import _assert_words

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
K = 4096


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    from paper_1604_01879_amd import _lib
    return _lib


@pytest.fixture(scope="module")
def case():
    """256 shapes x 64 views x 4096-d (40 classes, 20 % distractor views),
    8 queries of 20..64 views, a codebook of 4096 seeded database rows, and
    the oracle's MA = 3 words of every database view (its first column is
    the MA = 1 word: the order is (distance, index))."""
    _say("full-width case: generating and running the oracle quantizer")
    w = synth.PRESETS["c1"].scaled(n_shapes=256, dim=4096, n_queries=8, m_lo=20, m_hi=64,
                                   p_dis=0.2, seed=7)
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    cb = db[synth.kmeans_init_idx(db.shape[0], K, 11)]
    W3 = O.assign(db, cb, 3)
    qw = O.assign(q, cb, 1)[:, 0]
    return w, db, q, qoff, cb, W3, qw


def _views(L, db, nv, dtype):
    master = torch.from_numpy(db).to(DEV)
    if dtype == L.F32:
        return L.Views(master, nv, L.F32)
    codes, scale = L.gift_quantize_views(master, dtype)
    return L.Views(codes, nv, dtype, scale, master)


@pytest.mark.parametrize("ma", [1, 3])
def test_fullwidth_assign_and_lists(L, case, ma):
    w, db, q, qoff, cb, W3, qw = case
    _say(f"full-width assign + lists ma={ma}")
    cbt = torch.from_numpy(cb).to(DEV)
    words, unc = L.gift_assign(torch.from_numpy(db).to(DEV), cbt, ma)
    torch.cuda.synchronize()
    assert int(unc.item()) == 0
    _assert_words(words.cpu().numpy(), db, cb, ma)
    qwg, _ = L.gift_assign(torch.from_numpy(q).to(DEV), cbt, 1)
    _assert_words(qwg.cpu().numpy(), q, cb, 1)
    F = L.gift_build_fif(L.Views(torch.from_numpy(db).to(DEV), w.n_views, L.F32), cbt, ma)
    torch.cuda.synchronize()
    off, es, ev = O.build_fif(W3[:, :ma], K, w.n_views)
    assert np.array_equal(F.offsets.cpu().numpy(), off)
    assert np.array_equal(F.entry_shape.cpu().numpy(), es)
    assert np.array_equal(F.entry_view.cpu().numpy(), ev)


@pytest.mark.parametrize("dtype_name", ["f32", "fp8"])
def test_fullwidth_exhaustive_ranked_ids(L, case, dtype_name):
    w, db, q, qoff, cb, W3, qw = case
    _say(f"full-width exhaustive {dtype_name}")
    dt = {"f32": L.F32, "fp8": L.FP8E4M3}[dtype_name]
    V = _views(L, db, w.n_views, dt)
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    k, R = 20, 60
    ids, sc, fl = L.gift_query_exhaustive(V, Q, k, R)
    torch.cuda.synchronize()
    ids, sc, fl = ids.cpu().numpy(), sc.cpu().numpy(), fl.cpu().numpy()
    S = O.exhaustive_scores(q, qoff, db, w.n_views)
    if dtype_name == "f32":
        S1 = S
    else:
        qc, qs = O.quantize_views(q, dtype_name)
        dc, ds = O.quantize_views(db, dtype_name)
        S1 = O.lowprec_exhaustive_scores(qc, qs, qoff, dc, ds, w.n_views)
    for b in range(len(qoff) - 1):
        assert_returned_exact(ids[b], sc[b], S[b], k)
        if dtype_name == "f32" or fl[b] & 1:
            assert_ranked_equal(ids[b], sc[b], S[b], k)
    assert_flags_as_predicted(fl, S1, S, qoff, R, k, dtype_name, w.dim)
    if dtype_name == "f32":
        assert fl.all()


@pytest.mark.parametrize("dtype_name", ["f32", "fp8"])
@pytest.mark.parametrize("ma", [1, 3])
def test_fullwidth_fif_ranked_ids(L, case, dtype_name, ma):
    w, db, q, qoff, cb, W3, qw = case
    _say(f"full-width F-IF {dtype_name} ma={ma}")
    dt = {"f32": L.F32, "fp8": L.FP8E4M3}[dtype_name]
    master = torch.from_numpy(db).to(DEV)
    F = L.gift_build_fif(L.Views(master, w.n_views, L.F32), torch.from_numpy(cb).to(DEV), ma)
    V = _views(L, db, w.n_views, dt)
    Q = L.Queries(torch.from_numpy(q).to(DEV), torch.from_numpy(qoff))
    k, R = 20, 60
    ids, sc, fl = L.gift_query_fif(V, F, Q, k, R)
    torch.cuda.synchronize()
    ids, sc, fl = ids.cpu().numpy(), sc.cpu().numpy(), fl.cpu().numpy()
    off, es, ev = O.build_fif(W3[:, :ma], K, w.n_views)
    S = O.fif_scores(q, qoff, db, w.n_views, cb, off, es, ev, qwords=qw)
    assert (fl >> 1 == 0).all()  # every query word certified
    for b in range(len(qoff) - 1):
        assert_returned_exact(ids[b], sc[b], S[b], k)
        if dtype_name == "f32" or fl[b] & 1:
            assert_ranked_equal(ids[b], sc[b], S[b], k)
    if dtype_name == "f32":
        S1 = S
    else:
        qc, qs = O.quantize_views(q, dtype_name)
        dc, ds = O.quantize_views(db, dtype_name)
        S1 = O.fif_scores(O.dequantize(qc, qs), qoff, O.dequantize(dc, ds), w.n_views, cb,
                          off, es, ev, qwords=qw)
    assert_flags_as_predicted(fl, S1, S, qoff, R, k, dtype_name, w.dim, list_scan=True)
