"""Writes the float64 Eq. 3 reference ranking of the 12,000-shape precision
workload: the exact top-100 of all 256 queries (12,000 shapes x 64 views x
4096-d database, 256 queries x 64 views, seed 0).

Calls only ``oracle/`` (the float64 Eq. 3 scores, Sec. 2.3, and the ranking
by score descending, id ascending) and ``synth/`` (the seeded inputs).  It runs
on the CPU (about 15 minutes on 8 cores) and writes
``tests/golden/c3_fp64_top100.npz`` with

* ``ids``    int32   [256, 100]  the float64 top-100 shape ids per query;
* ``scores`` float64 [256, 100]  their Eq. 3 scores, evaluated in float64
  over the float32 inputs;
* ``next``   float64 [256]       the 101st best score (the margin of the
  100th);
* ``q_sha256``, ``db_probe_sha256``: digests of the query views and of every
  1,000th database row, so a reader can check that its inputs are the same.

Usage: python tests/golden/make_c3_fp64_topk.py [out.npz]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import synth  # noqa: E402

TOP = 100


def input_digests(db: np.ndarray, q: np.ndarray):
    """sha256 of the query views and of database rows 0, 1000, 2000, ..."""
    qd = hashlib.sha256(np.ascontiguousarray(q).tobytes()).hexdigest()
    dd = hashlib.sha256(np.ascontiguousarray(db[::1000]).tobytes()).hexdigest()
    return qd, dd


def main(out_path: str) -> None:
    w = synth.PRESETS["c3"]
    t0 = time.time()
    db, _, _ = synth.make_db(w)
    q, qoff, _ = synth.make_queries(w)
    print(f"inputs {db.shape} + {q.shape} in {time.time() - t0:.0f} s", flush=True)
    S = np.empty((w.n_queries, w.n_shapes), np.float64)
    # Eq. 3 in float64, 32 queries at a time (progress lines in between)
    for b0 in range(0, w.n_queries, 32):
        b1 = min(w.n_queries, b0 + 32)
        lo, hi = int(qoff[b0]), int(qoff[b1])
        S[b0:b1] = O.exhaustive_scores(q[lo:hi], qoff[b0:b1 + 1] - lo, db, w.n_views)
        print(f"queries {b1}/{w.n_queries} at {time.time() - t0:.0f} s", flush=True)
    ids, sc = O.rank_topk(S, TOP + 1)
    qd, dd = input_digests(db, q)
    np.savez_compressed(out_path, ids=ids[:, :TOP].astype(np.int32), scores=sc[:, :TOP],
                        next=sc[:, TOP].copy(), q_sha256=np.array(qd),
                        db_probe_sha256=np.array(dd))
    print(f"wrote {out_path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1
         else os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_fp64_top100.npz"))
