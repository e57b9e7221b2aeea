"""Seeded synthetic inputs for the GIFT search stage.

The paper's features are CNN activations of rendered depth views, one
L2-normalised vector per view and 64 views per shape (Sec. 2.1, 2.2 and the
default setup at the start of Sec. 3).  Neither the datasets nor the trained
network are available, so every workload here is drawn from a seeded
class-structured generator with the same shapes:

* one Gaussian centre per class, ``mu_c ~ N(0, I_d)``;
* shape ``i`` belongs to class ``i mod C``;
* each view independently becomes a "distractor" with probability
  ``p_dis`` and then takes a uniformly chosen *other* class;
* a view is ``relu(mu_class + sigma * eps)``, L2-normalised with the norm
  taken in float64 and the result stored as float32 (non-negative, unit norm,
  as the paper's normalised activations are).

This module holds only random-number plumbing and the input recipe.  It
computes nothing of the search method itself, and is the one piece of code
shared by the CPU oracle and the GPU path.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, replace

import numpy as np

# Order in which child seed streams are spawned from SeedSequence(seed).
_STREAMS = ("centres", "db_classes", "db_noise", "q_classes", "q_counts",
            "q_noise", "kmeans_init", "arrivals", "subcentres", "centres2")
_CHUNK = 2048  # views per noise chunk; each chunk has its own seed


@dataclass(frozen=True)
class Workload:
    """One synthetic search workload (database + query batch)."""
    name: str
    n_shapes: int          # N
    n_classes: int         # C
    n_views: int           # Nv (views per database shape)
    dim: int               # d
    sigma: float           # per-coordinate noise scale
    p_dis: float           # probability that a view is a cross-class distractor
    n_queries: int         # B
    m_lo: int              # query view count range, inclusive
    m_hi: int
    K: int                 # codebook size
    ma: tuple              # multiple-assignment values exercised
    top_k: int
    seed: int = 0
    n_sub: int = 0         # per-class viewpoint sub-centres (0: none)
    sub_sigma: float = 0.5  # scale of the sub-centre offsets

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


# The five workloads, smallest first.
PRESETS = {
    # CPU-sized: 1,000 shapes x 64 views x 256-d, 8 queries, K=64, top-10.
    "c1": Workload("c1", 1000, 40, 64, 256, 0.3, 0.0, 8, 64, 64, 64, (1, 2), 10),
    # Plain FP32: 12,000 shapes (40 classes) x 64 x 4096, 20 % distractors,
    # K=4096, 256 queries x 64 views, MA in {1, 3}, top-100.
    "c2": Workload("c2", 12000, 40, 64, 4096, 0.3, 0.2, 256, 64, 64, 4096, (1, 3), 100),
    # Precision: the c2 database in BF16 / FP8 with FP32 rescore of top-200.
    "c3": Workload("c3", 12000, 40, 64, 4096, 0.3, 0.2, 256, 64, 64, 4096, (1,), 100),
    # Batching + S-IF: 50,000 shapes (100 classes), K=8192, 1,024 queries with
    # 12..64 views.
    "c4": Workload("c4", 50000, 100, 64, 4096, 0.3, 0.2, 1024, 12, 64, 8192, (1,), 100),
    # Serving: 200,000 shapes (200 classes) x 1024-d, 8..64 query views.
    "c5": Workload("c5", 200000, 200, 64, 1024, 0.3, 0.2, 1024, 8, 64, 8192, (1,), 100),
    # F-IF K x MA sweep (shape of the paper's Fig. 5): 4,096 shapes with 8
    # viewpoint sub-centres per class, 256-d, 256 queries, top-20.
    "sweep": Workload("sweep", 4096, 40, 64, 256, 0.3, 0.1, 256, 64, 64, 256, (1, 2, 3), 20,
                      0, 8, 0.8),
}


def _streams(seed: int) -> dict:
    children = np.random.SeedSequence(seed).spawn(len(_STREAMS))
    return dict(zip(_STREAMS, children))


def _threads(threads):
    if threads:
        return int(threads)
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def class_centres(w: Workload) -> np.ndarray:
    """Per-class centres mu_c ~ N(0, I_d), float32 [C, d]."""
    rng = np.random.Generator(np.random.PCG64(_streams(w.seed)["centres"]))
    return rng.standard_normal((w.n_classes, w.dim), dtype=np.float32)


def subcentre_offsets(w: Workload) -> np.ndarray:
    """Per (class, viewpoint) offsets nu ~ sub_sigma * N(0, I_d), float32
    [C, n_sub, d]: view j of a shape is drawn around mu_class + nu[class,
    j mod n_sub], so views taken from the same viewpoint agree across the
    shapes of a class (the structure an inverted file can exploit)."""
    rng = np.random.Generator(np.random.PCG64(_streams(w.seed)["subcentres"]))
    nu = rng.standard_normal((w.n_classes, max(1, w.n_sub), w.dim), dtype=np.float32)
    return (nu * np.float32(w.sub_sigma)).astype(np.float32)


def _centre_table(w: Workload):
    """Centres indexed by class * n_sub + viewpoint (or by class alone)."""
    mu = class_centres(w)
    if w.n_sub <= 0:
        return mu
    nu = subcentre_offsets(w)
    return (mu[:, None, :] + nu).reshape(w.n_classes * w.n_sub, w.dim)


def _view_classes(rng, base_cls: np.ndarray, n_views: int, C: int, p_dis: float):
    """Per-view class: the owner's class, or with prob. p_dis another class."""
    vc = np.repeat(base_cls.astype(np.int32), n_views)
    if p_dis > 0 and C > 1:
        dis = rng.random(vc.shape[0]) < p_dis
        shift = rng.integers(1, C, size=vc.shape[0], dtype=np.int32)
        vc = np.where(dis, (vc + shift) % C, vc).astype(np.int32)
    return vc


def _fill_views(out: np.ndarray, vclass: np.ndarray, centres: np.ndarray,
                sigma: float, seed: int, stream: int, threads) -> None:
    """out[v] = normalise(relu(centres[vclass[v]] + sigma * eps_v)).

    Noise for views [c*_CHUNK, (c+1)*_CHUNK) comes from
    SeedSequence([seed, stream, c]), so the result does not depend on the
    thread count or on chunk scheduling.
    """
    n = out.shape[0]
    nchunks = (n + _CHUNK - 1) // _CHUNK

    def work(c):
        lo, hi = c * _CHUNK, min(n, (c + 1) * _CHUNK)
        rng = np.random.Generator(np.random.PCG64(
            np.random.SeedSequence([seed, stream, c])))
        y = rng.standard_normal((hi - lo, out.shape[1]), dtype=np.float32)
        y *= np.float32(sigma)
        y += centres[vclass[lo:hi]]
        np.maximum(y, 0, out=y)
        y64 = y.astype(np.float64)
        nrm = np.sqrt(np.einsum("ij,ij->i", y64, y64))
        dead = nrm == 0
        if dead.any():  # an all-zero view after ReLU: use the first axis
            y64[dead, 0] = 1.0
            nrm[dead] = 1.0
        out[lo:hi] = (y64 / nrm[:, None]).astype(np.float32)

    with ThreadPoolExecutor(_threads(threads)) as ex:
        list(ex.map(work, range(nchunks)))


def make_db(w: Workload, out: np.ndarray | None = None, threads=None):
    """Database views, float32 [N*Nv, d] (shape-major), plus labels.

    Returns (views, shape_class int32 [N], view_class int32 [N*Nv]).
    ``out`` may be a preallocated float32 array (e.g. pinned host memory).
    """
    st = _streams(w.seed)
    centres = _centre_table(w)
    shape_cls = (np.arange(w.n_shapes) % w.n_classes).astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(st["db_classes"]))
    vclass = _view_classes(rng, shape_cls, w.n_views, w.n_classes, w.p_dis)
    nv = w.n_shapes * w.n_views
    if out is None:
        out = np.empty((nv, w.dim), dtype=np.float32)
    assert out.shape == (nv, w.dim) and out.dtype == np.float32
    rows = vclass
    if w.n_sub > 0:
        vpt = (np.arange(nv) % w.n_views) % w.n_sub
        rows = (vclass * w.n_sub + vpt).astype(np.int32)
    _fill_views(out, rows, centres, w.sigma, w.seed, 1, threads)
    return out, shape_cls, vclass


def query_counts(w: Workload) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(_streams(w.seed)["q_counts"]))
    if w.m_lo == w.m_hi:
        return np.full(w.n_queries, w.m_lo, dtype=np.int32)
    return rng.integers(w.m_lo, w.m_hi + 1, size=w.n_queries, dtype=np.int32)


def _query_labels(w: Workload):
    """Query classes [B], view counts [B], offsets [B+1] and per-view classes."""
    st = _streams(w.seed)
    rng = np.random.Generator(np.random.PCG64(st["q_classes"]))
    qcls = rng.integers(0, w.n_classes, size=w.n_queries, dtype=np.int32)
    counts = query_counts(w)
    offsets = np.zeros(w.n_queries + 1, dtype=np.int32)
    np.cumsum(counts, out=offsets[1:])
    vclass = np.repeat(qcls, counts)
    if w.p_dis > 0 and w.n_classes > 1:
        dis = rng.random(vclass.shape[0]) < w.p_dis
        shift = rng.integers(1, w.n_classes, size=vclass.shape[0], dtype=np.int32)
        vclass = np.where(dis, (vclass + shift) % w.n_classes, vclass).astype(np.int32)
    return qcls, counts, offsets, vclass


def make_queries(w: Workload, threads=None):
    """Fresh query shapes drawn from the same generator on separate streams.

    Returns (views float32 [sum m, d], offsets int32 [B+1], classes int32 [B]).
    """
    centres = _centre_table(w)
    qcls, counts, offsets, vclass = _query_labels(w)
    out = np.empty((int(offsets[-1]), w.dim), dtype=np.float32)
    rows = vclass
    if w.n_sub > 0:
        vpt = (np.arange(int(offsets[-1])) - np.repeat(offsets[:-1], counts)) % w.n_sub
        rows = (vclass * w.n_sub + vpt).astype(np.int32)
    _fill_views(out, rows, centres, w.sigma, w.seed, 2, threads)
    return out, offsets, qcls


def make_second_measure(w: Workload, dim: int = 256, sigma: float = 0.45, threads=None):
    """Features of the same database and query views under a second
    similarity measure, standing in for a second CNN layer (the paper fuses
    two, Sec. 2.4 and 3).  The views keep their classes and distractor
    pattern (they are the same rendered views), while the measure has its own
    class centres (stream "centres2"), its own noise streams and a larger
    noise scale, so it ranks less sharply than the first.

    Returns (db views float32 [N*Nv, dim], query views float32 [sum m, dim],
    query offsets int32 [B+1]).
    """
    st = _streams(w.seed)
    rng = np.random.Generator(np.random.PCG64(st["centres2"]))
    centres = rng.standard_normal((w.n_classes, dim), dtype=np.float32)
    shape_cls = (np.arange(w.n_shapes) % w.n_classes).astype(np.int32)
    vrng = np.random.Generator(np.random.PCG64(st["db_classes"]))
    vclass = _view_classes(vrng, shape_cls, w.n_views, w.n_classes, w.p_dis)
    db = np.empty((w.n_shapes * w.n_views, dim), dtype=np.float32)
    _fill_views(db, vclass, centres, sigma, w.seed, 3, threads)
    _, _, offsets, qvclass = _query_labels(w)
    q = np.empty((int(offsets[-1]), dim), dtype=np.float32)
    _fill_views(q, qvclass, centres, sigma, w.seed, 4, threads)
    return db, q, offsets


def kmeans_init_idx(n_train: int, K: int, seed: int) -> np.ndarray:
    """K distinct training-row indices from a seeded permutation (int64)."""
    if K > n_train:
        raise ValueError("K larger than the training set")
    rng = np.random.Generator(np.random.PCG64(_streams(seed)["kmeans_init"]))
    return np.sort(rng.permutation(n_train)[:K]).astype(np.int64)


def training_sample(n_total: int, n_sample: int, seed: int) -> np.ndarray:
    """Seeded sorted subset of view rows used to train a codebook."""
    if n_sample >= n_total:
        return np.arange(n_total, dtype=np.int64)
    ss = np.random.SeedSequence([seed, 7])
    rng = np.random.Generator(np.random.PCG64(ss))
    return np.sort(rng.choice(n_total, size=n_sample, replace=False)).astype(np.int64)


def poisson_arrivals(rate_qps: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a seeded Poisson process on [0, duration)."""
    rng = np.random.Generator(np.random.PCG64(_streams(seed)["arrivals"]))
    n_max = int(rate_qps * duration_s * 1.5 + 50)
    t = np.cumsum(rng.exponential(1.0 / rate_qps, size=n_max))
    return t[t < duration_s]
