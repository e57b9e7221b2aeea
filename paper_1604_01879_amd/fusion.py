"""Search with two similarity measures fused before the re-ranking.

The paper builds one sparse activation per shape and measure from its
neighbour list (Sec. 2.4, Eq. 7), replaces each measure's activation by its
mean over the top-k2 neighbours found by the other measure (neighbour
co-augmentation, Sec. 2.4.1, Eq. 11), fuses the two with the generalised
mean of exponent alpha (Eq. 9; alpha = 0.5 in every experiment of Sec. 3)
and re-ranks by Eq. 8 through the second inverted file built from the fused
activations (Eq. 13, 14).

Only the order of the library calls lives here; every step runs in libgift:
gift_query_exhaustive (Eq. 3 neighbour lists), gift_augment_neighbours
(Eq. 10 / 11), gift_fuse_activations (Eq. 9), gift_fuse_self (the fused self
membership of a query outside the database), gift_build_sif and
gift_rerank_sif (Eq. 7, 8, 13, 14).
"""
from __future__ import annotations

import torch

from . import _lib as L


def _query_rows(V: L.Views):
    """Float32 rows of the database views (the views themselves as queries)."""
    return V.master if V.master is not None else V.data


class TwoMeasureIndex:
    """The fused second inverted file of a database seen through two
    measures (two Views of the same shapes, e.g. two feature layers).

    Build: each database shape is queried against the database under each
    measure for its exact top-k1 by Eq. 3 (itself first); measure 1's rows
    are averaged over measure 2's top-k2 and the reverse (Eq. 11); the two
    are fused (Eq. 9) and indexed (Eq. 7, the S-IF).  rescore_r candidates
    are rescored exactly per neighbour query (see gift_query_exhaustive).
    """

    def __init__(self, V1: L.Views, V2: L.Views, k1=20, k2=4, alpha=0.5, rescore_r=None,
                 chunk=256, stream=None):
        if V1.n_shapes != V2.n_shapes or V1.n_views != V2.n_views:
            raise ValueError("the two measures must describe the same shapes and views")
        if not (1 <= k2 <= k1 <= V1.n_shapes):
            raise ValueError("need 1 <= k2 <= k1 <= n_shapes")
        self.V = (V1, V2)
        self.k1, self.k2, self.alpha = int(k1), int(k2), float(alpha)
        n = V1.n_shapes
        self.R = int(rescore_r or min(n, max(4 * k1, 64)))
        self.stream = stream
        self.nbr = [self._database_lists(V, chunk) for V in self.V]
        (i1, s1), (i2, s2) = self.nbr
        a1i, a1s, _ = L.gift_augment_neighbours(i1, s1, i2[:, :k2].contiguous(), stream=stream)
        a2i, a2s, _ = L.gift_augment_neighbours(i2, s2, i1[:, :k2].contiguous(), stream=stream)
        self.rows = L.gift_fuse_activations(a1i, a1s, a2i, a2s, self.alpha, stream=stream)
        self.sif = L.gift_build_sif(*self.rows, stream=stream)

    def _database_lists(self, V: L.Views, chunk):
        """Exact top-k1 of every database shape under one measure."""
        rows = _query_rows(V)
        nv, n = V.n_views, V.n_shapes
        ids, scores = [], []
        for c0 in range(0, n, chunk):
            c1 = min(n, c0 + chunk)
            off = torch.arange(0, c1 - c0 + 1, dtype=torch.int32) * nv
            Q = L.Queries(rows[c0 * nv:c1 * nv], off, offsets_host=off)
            i, s, _ = L.gift_query_exhaustive(V, Q, self.k1, self.R, stream=self.stream)
            ids.append(i)
            scores.append(s)
        return torch.cat(ids).contiguous(), torch.cat(scores).contiguous()

    def query(self, Q1: L.Queries, Q2: L.Queries, top_k):
        """Fused re-ranking of a query batch given under both measures (the
        same query shapes): (ids [B, top_k], scores [B, top_k]).  Each query
        takes its top-(k1 - 1) under each measure plus itself (membership 1,
        the Eq. 3 self score of unit-norm views), is co-augmented over itself
        and its top-(k2 - 1) neighbours of the other measure, fused, and
        re-ranked by Eq. 8."""
        if Q1.n_queries != Q2.n_queries:
            raise ValueError("the two query batches must hold the same queries")
        k1, k2, st = self.k1, self.k2, self.stream
        V1, V2 = self.V
        qi1, qs1, _ = L.gift_query_exhaustive(V1, Q1, k1 - 1, self.R, stream=st)
        qi2, qs2, _ = L.gift_query_exhaustive(V2, Q2, k1 - 1, self.R, stream=st)
        (i1, s1), (i2, s2) = self.nbr
        if k2 > 1:
            m1, m2 = qi2[:, :k2 - 1].contiguous(), qi1[:, :k2 - 1].contiguous()
        else:  # no database member: the query's own list alone
            m1 = m2 = torch.full((Q1.n_queries, 1), -1, dtype=torch.int32, device=qi1.device)
        a1i, a1s, n1 = L.gift_augment_neighbours(i1, s1, m1, qi1, qs1, stream=st)
        a2i, a2s, n2 = L.gift_augment_neighbours(i2, s2, m2, qi2, qs2, stream=st)
        fi, fs = L.gift_fuse_activations(a1i, a1s, a2i, a2s, self.alpha, stream=st)
        one = torch.ones(Q1.n_queries, dtype=torch.float32, device=qi1.device)
        q_self = L.gift_fuse_self(one, n1, one, n2, self.alpha, stream=st)
        ids, scores, _ = L.gift_rerank_sif(self.sif, fi, fs, q_self, top_k, stream=st)
        return ids, scores
