"""Generator statistics and determinism (CPU)."""
import numpy as np

import synth


def _w(**kw):
    base = dict(n_shapes=80, dim=48, n_queries=6)
    base.update(kw)
    return synth.PRESETS["c1"].scaled(**base)


def test_unit_norm_nonnegative_and_classes():
    w = _w(p_dis=0.25)
    db, scls, vcls = synth.make_db(w)
    assert db.dtype == np.float32 and db.shape == (80 * 64, 48)
    assert (db >= 0).all()
    assert np.allclose(np.linalg.norm(db.astype(np.float64), axis=1), 1.0, atol=1e-6)
    assert (np.bincount(scls, minlength=40) == 2).all()
    rate = float((vcls != np.repeat(scls, 64)).mean())
    assert abs(rate - 0.25) < 0.03


def test_deterministic_across_thread_counts():
    w = _w()
    a, _, _ = synth.make_db(w, threads=1)
    b, _, _ = synth.make_db(w, threads=4)
    assert np.array_equal(a, b)
    q1 = synth.make_queries(w, threads=1)
    q2 = synth.make_queries(w, threads=3)
    for x, y in zip(q1, q2):
        assert np.array_equal(x, y)


def test_query_counts_range_and_offsets():
    w = _w(m_lo=8, m_hi=64, n_queries=200)
    q, off, cls = synth.make_queries(w)
    cnt = np.diff(off)
    assert cnt.min() >= 8 and cnt.max() <= 64 and len(set(cnt.tolist())) > 20
    assert q.shape[0] == off[-1]


def test_within_class_views_more_similar():
    w = _w()
    db, scls, vcls = synth.make_db(w)
    sim = db[:640].astype(np.float64) @ db[:640].T.astype(np.float64)
    same = vcls[:640, None] == vcls[None, :640]
    assert sim[same].mean() > sim[~same].mean() + 0.2


def test_kmeans_init_and_sample_and_arrivals():
    i = synth.kmeans_init_idx(1000, 64, 0)
    assert len(set(i.tolist())) == 64 and i.max() < 1000
    assert np.array_equal(i, synth.kmeans_init_idx(1000, 64, 0))
    s = synth.training_sample(10000, 500, 0)
    assert len(set(s.tolist())) == 500
    t = synth.poisson_arrivals(200.0, 10.0, 0)
    assert abs(len(t) - 2000) < 200 and (np.diff(t) > 0).all()


def test_subcentres_group_views_by_viewpoint():
    w = synth.PRESETS["c1"].scaled(n_shapes=80, dim=48, n_queries=4, n_sub=4, sub_sigma=1.0)
    db, scls, vcls = synth.make_db(w)
    assert np.allclose(np.linalg.norm(db.astype(np.float64), axis=1), 1.0, atol=1e-6)
    x = db.astype(np.float64)
    # shapes 0 and 40 share class 0: same-viewpoint views are closer than
    # other-viewpoint views of the same class
    a, b = x[0:64], x[40 * 64:41 * 64]
    sim = a @ b.T
    vp = np.arange(64) % 4
    same = vp[:, None] == vp[None, :]
    cls_ok = (vcls[0:64][:, None] == 0) & (vcls[40 * 64:41 * 64][None, :] == 0)
    assert sim[same & cls_ok].mean() > sim[~same & cls_ok].mean() + 0.05
    # without sub-centres the preset data is unchanged
    base, _, _ = synth.make_db(synth.PRESETS["c1"].scaled(n_shapes=10, dim=32))
    again, _, _ = synth.make_db(synth.PRESETS["c1"].scaled(n_shapes=10, dim=32, n_sub=0))
    assert np.array_equal(base, again)


def test_second_measure_same_views_own_features():
    """The second measure describes the same views: same query offsets, and
    views of one class (the first measure's labels) are closer to each other
    than to other classes' views; its features are deterministic, unit-norm
    and non-negative, and differ from the first measure's."""
    w = synth.PRESETS["c1"].scaled(n_shapes=80, dim=64, n_queries=5, m_lo=4, m_hi=12,
                                   p_dis=0.25, seed=3)
    db1, _, vclass = synth.make_db(w)
    _, qoff, _ = synth.make_queries(w)
    db2, q2, qoff2 = synth.make_second_measure(w, dim=48)
    again = synth.make_second_measure(w, dim=48)
    assert np.array_equal(db2, again[0]) and np.array_equal(q2, again[1])
    assert np.array_equal(qoff, qoff2) and q2.shape == (int(qoff[-1]), 48)
    assert db2.shape == (db1.shape[0], 48) and (db2 >= 0).all()
    assert np.allclose(np.linalg.norm(db2, axis=1), 1.0, atol=1e-6)
    G = db2[:1000].astype(np.float64) @ db2[:1000].T.astype(np.float64)
    same = vclass[:1000, None] == vclass[None, :1000]
    off_diag = ~np.eye(1000, dtype=bool)
    assert G[same & off_diag].mean() > G[~same].mean() + 0.1
