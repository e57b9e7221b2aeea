"""Continuous-batching query server over batch plans.

The index (database views, F-IF, optional S-IF) stays resident in HBM.  A
pool of plan slots (each a captured HIP graph with its own stream and
input/output buffers) serves arriving queries: whenever a slot is free, the
dispatcher admits pending requests in arrival order while they fit the
slot's query and view capacity, launches the slot's graph (and the S-IF
re-rank) on the slot's stream and moves on, so batches on different slots
overlap on the device.  The number of slots follows from a device-memory
budget.  Completed batches are detected by events and their requests
resolved with (ids, scores) and latency.

Only scheduling lives here; every step of the search runs in libgift.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future

import numpy as np
import torch

from . import _lib as L
from .sched import form_batch, slots_for_budget


class _Request:
    __slots__ = ("views", "m", "t_arrival", "future", "t_done")

    def __init__(self, views, t_arrival):
        self.views = views
        self.m = int(views.shape[0])
        self.t_arrival = t_arrival
        self.future = Future()
        self.t_done = None


class _Slot:
    def __init__(self, db, fif, sif, max_queries, max_views, max_m, fif_k, top_k, rescore_r):
        self.plan = L.FifPlan(db, fif, max_queries, max_views, max_m, fif_k, rescore_r)
        dev = db.data.device
        self.stream = self.plan.stream
        self.staging = torch.empty((max_views, db.dim), dtype=torch.float32).pin_memory()
        self.off_host = torch.zeros(max_queries + 1, dtype=torch.int32).pin_memory()
        self.sif = sif
        self.top_k = top_k
        if sif is not None:
            self.self_m = torch.ones(max_queries, dtype=torch.float32, device=dev)
            self.out_ids = torch.zeros((max_queries, top_k), dtype=torch.int32, device=dev)
            self.out_sc = torch.zeros((max_queries, top_k), dtype=torch.float32, device=dev)
            self.out_flags = torch.zeros(max_queries, dtype=torch.int32, device=dev)
        self.host_ids = torch.zeros((max_queries, top_k), dtype=torch.int32).pin_memory()
        self.host_sc = torch.zeros((max_queries, top_k), dtype=torch.float32).pin_memory()
        self.event = torch.cuda.Event()
        self.batch = None

    def launch(self, reqs):
        views = 0
        self.off_host[0] = 0
        for i, r in enumerate(reqs):
            self.staging[views:views + r.m].copy_(torch.from_numpy(r.views))
            views += r.m
            self.off_host[i + 1] = views
        n = len(reqs)
        with torch.cuda.stream(self.stream):
            self.plan.views[:views].copy_(self.staging[:views], non_blocking=True)
            self.plan.offsets[:n + 1].copy_(self.off_host[:n + 1], non_blocking=True)
        self.plan.run(n, views, stream=self.stream)
        if self.sif is not None:
            # re-rank with the batch's F-IF neighbours plus the query itself
            ids, sc = _rerank_into(self.sif, self.plan.ids[:n], self.plan.scores[:n],
                                   self.self_m[:n], self.top_k, self.stream,
                                   self.out_ids[:n], self.out_sc[:n], self.out_flags[:n])
        else:
            ids, sc = self.plan.ids[:n], self.plan.scores[:n]
        with torch.cuda.stream(self.stream):
            self.host_ids[:n].copy_(ids, non_blocking=True)
            self.host_sc[:n].copy_(sc, non_blocking=True)
            self.event.record(self.stream)
        self.batch = reqs

    def poll(self):
        if self.batch is None or not self.event.query():
            return None
        reqs, self.batch = self.batch, None
        return reqs

    def close(self):
        self.plan.close()


def _rerank_into(sif, q_ids, q_sc, self_m, top_k, stream, out_ids, out_sc, flags):
    """gift_rerank_sif on `stream` into buffers owned by the slot."""
    import ctypes as C
    B, k1 = q_ids.shape
    L._check(L._lib.gift_rerank_sif(sif.n_shapes, L._ptr(sif.l1), L._ptr(sif.post_off),
                                    L._ptr(sif.post_id), L._ptr(sif.post_val), B, k1,
                                    L._ptr(q_ids), L._ptr(q_sc), L._ptr(self_m), top_k,
                                    L._ptr(out_ids), L._ptr(out_sc), L._ptr(flags),
                                    C.c_void_p(stream.cuda_stream)))
    return out_ids, out_sc


class Server:
    """Continuous-batching search over a resident index.

    With `sif`, each query takes its top-(k1 - 1) by Eq. 4 plus itself (S-IF
    self membership 1, the Eq. 3 self score of unit-norm views) and is
    re-ranked by Eq. 8; otherwise the Eq. 4 ranking is returned.
    """

    def __init__(self, db, fif, sif=None, top_k=100, k1=20, rescore_r=200, max_queries=64,
                 max_views=64 * 64, max_m=64, mem_budget_bytes=None, max_slots=3):
        fif_k = (k1 - 1) if sif is not None else top_k
        probe = L._lib.gift_fif_plan_workspace(
            __import__("ctypes").byref(db.c), __import__("ctypes").byref(fif.c), max_queries,
            max_views, fif_k, rescore_r)
        per_slot = int(probe) + max_views * db.dim * 4
        self.n_slots = slots_for_budget(per_slot, mem_budget_bytes, max_slots)
        self.slots = [_Slot(db, fif, sif, max_queries, max_views, max_m, fif_k, top_k,
                            max(rescore_r, fif_k)) for _ in range(self.n_slots)]
        self.max_queries, self.max_views, self.max_m = max_queries, max_views, max_m
        self.dim = db.dim
        self.pending = collections.deque()
        self.lock = threading.Condition()
        self.stop = False
        self.batches = 0
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    def submit(self, views):
        """Queues one query (float32 [m, dim] host array); returns a Future of
        (ids, scores, latency seconds)."""
        views = np.ascontiguousarray(views, dtype=np.float32)
        if views.ndim != 2 or views.shape[1] != self.dim:
            raise ValueError("query views must be [m, dim]")
        if views.shape[0] < 1 or views.shape[0] > min(self.max_m, self.max_views):
            raise ValueError("query view count outside the server's capacity")
        r = _Request(views, time.perf_counter())
        with self.lock:
            self.pending.append(r)
            self.lock.notify()
        return r.future

    def _loop(self):
        while True:
            launched = False
            for s in self.slots:
                done = s.poll()
                if done is not None:
                    t = time.perf_counter()
                    n = len(done)
                    ids = s.host_ids[:n].numpy().copy()
                    sc = s.host_sc[:n].numpy().copy()
                    for i, r in enumerate(done):
                        r.future.set_result((ids[i], sc[i], t - r.t_arrival))
                if s.batch is None:
                    with self.lock:
                        n = form_batch((r.m for r in self.pending), self.max_queries,
                                       self.max_views)
                        reqs = [self.pending.popleft() for _ in range(n)]
                    if reqs:
                        s.launch(reqs)
                        self.batches += 1
                        launched = True
            with self.lock:
                if self.stop and not self.pending and all(s.batch is None for s in self.slots):
                    return
                if not launched and not any(s.batch is not None for s in self.slots):
                    if not self.pending and not self.stop:
                        self.lock.wait(timeout=0.05)
            if not launched:
                time.sleep(0.0002)

    def close(self):
        with self.lock:
            self.stop = True
            self.lock.notify()
        self.thread.join()
        for s in self.slots:
            s.close()


def replay_trace(server, queries, arrivals):
    """Submits queries[i] at time arrivals[i] (seconds from now); waits for all
    and returns (results list, latencies array, wall seconds)."""
    t0 = time.perf_counter()
    futs = []
    for v, t in zip(queries, arrivals):
        delay = t0 + t - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        futs.append(server.submit(v))
    res = [f.result() for f in futs]
    wall = time.perf_counter() - t0
    lat = np.array([r[2] for r in res])
    return res, lat, wall
