"""Continuous-batching query server over batch plans, admitted by memory.

The index (database views, F-IF, optional S-IF) stays resident in HBM.
Queries arrive one at a time; a dispatcher forms batches from the pending
queries in arrival order and runs each batch on a plan slot: a captured HIP
graph (the persistent first-pass kernel, selection, exact rescore and
ranking) with its own stream and buffers, followed by the S-IF re-rank.
Batches on different slots overlap on the device.

Memory admission: every slot's device memory (its plan workspace and its
query-view buffer) is carved from one arena of `mem_budget_bytes`.  Slots
come in a few capacity classes (1, 4, 16, ... queries of up to max_m views
each).  A batch goes to an idle slot that holds it; otherwise a slot of the
smallest class that holds it is created in free arena memory, evicting idle
slots when the arena is full; when neither is possible the queries wait
until a running batch completes and its slot becomes idle.

Completion is event driven: each slot has a thread that blocks on the
slot's completion event, resolves the batch's futures with (ids, scores,
latency) and wakes the dispatcher.

Only scheduling lives here; every step of the search runs in libgift.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from concurrent.futures import Future

import numpy as np
import torch

from . import _lib as L
from .sched import Arena, form_batch, pick_class


class _Request:
    __slots__ = ("views", "m", "t_arrival", "future")

    def __init__(self, views, t_arrival):
        self.views = views
        self.m = int(views.shape[0])
        self.t_arrival = t_arrival
        self.future = Future()


class _Slot:
    """One plan with its stream, buffers carved from the server's arena and
    a completion thread."""

    def __init__(self, srv, cls, off):
        self.srv, self.cls, self.off = srv, cls, off
        q_cap, v_cap = srv.classes[cls]
        self.q_cap, self.v_cap = q_cap, v_cap
        ws_bytes = srv.ws_bytes[cls]
        buf = srv.arena_buf
        ws = buf[off:off + ws_bytes]
        v_off = off + (ws_bytes + 255) // 256 * 256
        views = buf[v_off:v_off + v_cap * srv.dim * 4].view(torch.float32).view(v_cap, srv.dim)
        self.plan = L.FifPlan(srv.db, srv.fif, q_cap, v_cap, srv.max_m, srv.fif_k, srv.rescore_r,
                              ws=ws, views=views, **srv.tuning)
        self.stream = self.plan.stream
        dev = srv.db.data.device
        self.staging = torch.empty((v_cap, srv.dim), dtype=torch.float32).pin_memory()
        self.off_host = torch.zeros(q_cap + 1, dtype=torch.int32).pin_memory()
        # numpy views of the pinned buffers: filling them costs a memcpy,
        # not a torch call per query (about 90 us for one query through torch)
        self.staging_np = self.staging.numpy()
        self.off_np = self.off_host.numpy()
        k = srv.top_k
        if srv.sif is not None:
            self.self_m = torch.ones(q_cap, dtype=torch.float32, device=dev)
            self.out_ids = torch.zeros((q_cap, k), dtype=torch.int32, device=dev)
            self.out_sc = torch.zeros((q_cap, k), dtype=torch.float32, device=dev)
            self.out_flags = torch.zeros(q_cap, dtype=torch.int32, device=dev)
            self.host_flags = torch.zeros(q_cap, dtype=torch.int32).pin_memory()
        self.host_ids = torch.zeros((q_cap, k), dtype=torch.int32).pin_memory()
        self.host_sc = torch.zeros((q_cap, k), dtype=torch.float32).pin_memory()
        # the arguments of gift_fif_plan_serve that do not change per batch
        sp = self.stream.cuda_stream
        self.serve_head = (self.plan.handle, self.staging.data_ptr(), self.off_host.data_ptr())
        if srv.sif is not None:
            sif = srv.sif
            self.serve_tail = (sif.n_shapes, sif.l1.data_ptr(), sif.post_off.data_ptr(),
                               sif.post_id.data_ptr(), sif.post_val.data_ptr(),
                               self.self_m.data_ptr(), k, self.out_ids.data_ptr(),
                               self.out_sc.data_ptr(), self.out_flags.data_ptr(),
                               self.host_ids.data_ptr(), self.host_sc.data_ptr(),
                               self.host_flags.data_ptr(), sp)
        else:
            self.serve_tail = (0, None, None, None, None, None, 0, None, None, None,
                               self.host_ids.data_ptr(), self.host_sc.data_ptr(), None, sp)
        self.event = torch.cuda.Event(blocking=True)
        self.busy = False
        self.last_used = 0.0
        self.jobs = queue.Queue()
        self.thread = threading.Thread(target=self._complete, daemon=True)
        self.thread.start()

    def launch(self, reqs):
        self.busy = True
        views = 0
        self.off_np[0] = 0
        for i, r in enumerate(reqs):
            self.staging_np[views:views + r.m] = r.views
            views += r.m
            self.off_np[i + 1] = views
        n = len(reqs)
        # copies in, the plan, the re-rank with the batch's F-IF neighbours
        # plus the query itself, copies out: one library call
        L.fif_plan_serve(*self.serve_head, n, views, *self.serve_tail)
        self.event.record(self.stream)
        self.jobs.put(reqs)

    def _complete(self):
        while True:
            reqs = self.jobs.get()
            if reqs is None:
                return
            self.event.synchronize()
            t = time.perf_counter()
            n = len(reqs)
            ids = self.host_ids[:n].numpy().copy()
            sc = self.host_sc[:n].numpy().copy()
            multi = int((self.host_flags[:n].numpy() & 2 != 0).sum()) if self.srv.sif is not None \
                else 0
            for i, r in enumerate(reqs):
                r.future.set_result((ids[i], sc[i], t - r.t_arrival))
            self.srv._done(self, multi)

    def close(self):
        self.jobs.put(None)
        self.thread.join()
        self.plan.close()


class Server:
    """Continuous-batching search over a resident index, admitted by memory.

    With `sif`, each query takes its top-(k1 - 1) by Eq. 4 plus itself (S-IF
    self membership 1, the Eq. 3 self score of unit-norm views) and is
    re-ranked by Eq. 8; otherwise the Eq. 4 ranking is returned.
    max_queries / max_m: the largest batch and the most views of one query.
    mem_budget_bytes (default: room for max_slots slots of the largest
    class) is the arena every slot is carved from; max_slots bounds the
    number of slots (streams).  prewarm creates slots of the largest class
    that fits while the budget and max_slots allow, so no graph is captured
    while queries wait.  tuning: the plans' settings (blocks_per_cu,
    list_tile, narrow_max; e.g. from tune.tune_plan), default the library's.
    """

    def __init__(self, db, fif, sif=None, top_k=100, k1=20, rescore_r=200, max_queries=64,
                 max_m=64, mem_budget_bytes=None, max_slots=3, prewarm=True, tuning=None):
        self.db, self.fif, self.sif = db, fif, sif
        self.tuning = dict(tuning or {})
        self.top_k, self.max_m, self.dim = top_k, max_m, db.dim
        self.fif_k = (k1 - 1) if sif is not None else top_k
        self.rescore_r = max(rescore_r, self.fif_k)
        qs = sorted({q for q in (1, 4, 16, max_queries) if q <= max_queries})
        self.classes = [(q, q * max_m) for q in qs]
        t = L.plan_tuning(**self.tuning)
        self.ws_bytes = [L.fif_plan_workspace(db, fif, q, v, self.fif_k, self.rescore_r, t)
                         for q, v in self.classes]
        self.slot_bytes = [(w + 255) // 256 * 256 + v * db.dim * 4
                           for w, (q, v) in zip(self.ws_bytes, self.classes)]
        if mem_budget_bytes is None:
            mem_budget_bytes = max_slots * (self.slot_bytes[-1] + 256)
        if mem_budget_bytes < self.slot_bytes[0]:
            raise ValueError(f"memory budget {mem_budget_bytes} below one slot of the smallest "
                             f"class ({self.slot_bytes[0]} bytes)")
        self.arena = Arena(mem_budget_bytes)
        self.arena_buf = torch.empty(mem_budget_bytes, dtype=torch.uint8, device=db.data.device)
        self.max_slots = max_slots
        self.slots = []
        self.pending = collections.deque()
        self.cond = threading.Condition()
        self.stop = False
        self.stats = {"batches": 0, "slots_created": 0, "slots_evicted": 0, "memory_waits": 0,
                      "max_busy_slots": 0, "multi_range_reranks": 0, "peak_bytes": 0}
        if prewarm:
            with self.cond:
                while len(self.slots) < max_slots:
                    cls = max((c for c in range(len(self.classes))
                               if self.arena.largest_free() >= self.slot_bytes[c]), default=None)
                    if cls is None:
                        break
                    self._create(cls)
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    # ------------------------------------------------------------ slots
    def _create(self, cls):
        off = self.arena.alloc(self.slot_bytes[cls])
        if off is None:
            return None
        s = _Slot(self, cls, off)
        self.slots.append(s)
        self.stats["slots_created"] += 1
        self.stats["peak_bytes"] = max(self.stats["peak_bytes"], self.arena.in_use())
        return s

    def _evict(self, s):
        self.slots.remove(s)
        s.close()
        self.arena.release(s.off)
        self.stats["slots_evicted"] += 1

    def _room_after_evicting(self, idle, cls):
        """Whether evicting every idle slot could free room for a slot of
        class cls (bytes and slot count; the arena may still be too
        fragmented, which _make checks)."""
        free = sum(length for _, length in self.arena.free)
        freed = sum(self.slot_bytes[s.cls] for s in idle)
        return free + freed >= self.slot_bytes[cls] and \
            len(self.slots) - len(idle) < self.max_slots

    def _make(self, cls, idle):
        """A new slot of class cls, evicting idle slots (least recently used
        first) only until it fits; None if it does not."""
        for victim in sorted(idle, key=lambda s: s.last_used):
            if len(self.slots) < self.max_slots and \
                    self.arena.largest_free() >= self.slot_bytes[cls]:
                break
            self._evict(victim)
        if len(self.slots) >= self.max_slots:
            return None
        return self._create(cls)

    def _slot_for(self, n, v):
        """(slot, n) for the leading n pending queries (v views), n possibly
        reduced to what the slot holds; (None, 0) when every slot is busy and
        memory holds no new one, so the queries wait.  In order: an idle slot
        that holds the batch; a new slot of the smallest class that holds
        it, if free memory (plus idle slots worth evicting) has room; the
        largest idle slot with the batch cut to fit; a new slot of the
        largest class that fits in free memory, batch cut to fit."""
        idle = [s for s in self.slots if not s.busy]
        fit = [s for s in idle if n <= s.q_cap and v <= s.v_cap]
        if fit:
            return min(fit, key=lambda s: (s.q_cap, s.last_used)), n
        cls = pick_class(n, v, self.classes)
        if cls is not None and self._room_after_evicting(idle, cls):
            s = self._make(cls, idle)
            if s is not None:
                return s, n
            idle = [s for s in self.slots if not s.busy]
        if idle:
            s = max(idle, key=lambda s: s.q_cap)
            return s, -1
        if len(self.slots) < self.max_slots:
            for c in range(len(self.classes) - 1, -1, -1):
                if self.arena.largest_free() >= self.slot_bytes[c]:
                    return self._create(c), -1
        return None, 0

    def _done(self, slot, multi):
        with self.cond:
            slot.busy = False
            slot.last_used = time.perf_counter()
            self.stats["multi_range_reranks"] += multi
            self.cond.notify_all()

    # ------------------------------------------------------------ requests
    def submit(self, views):
        """Queues one query (float32 [m, dim] host array); returns a Future of
        (ids, scores, latency seconds)."""
        views = np.ascontiguousarray(views, dtype=np.float32)
        if views.ndim != 2 or views.shape[1] != self.dim:
            raise ValueError("query views must be [m, dim]")
        if views.shape[0] < 1 or views.shape[0] > self.max_m:
            raise ValueError("query view count outside the server's capacity")
        r = _Request(views, time.perf_counter())
        with self.cond:
            self.pending.append(r)
            self.cond.notify_all()
        return r.future

    def _dispatch(self):
        """Launches batches while queries are pending and a slot can take
        them; returns when none can.  Called with the lock held."""
        q_max, v_max = self.classes[-1]
        while self.pending:
            n = form_batch((r.m for r in self.pending), q_max, v_max)
            v = sum(r.m for r in list(self.pending)[:n])
            slot, n = self._slot_for(n, v)
            if slot is None:
                self.stats["memory_waits"] += 1
                return
            if n < 0:  # the slot holds only a leading part of the batch
                n = form_batch((r.m for r in self.pending), slot.q_cap, slot.v_cap)
            reqs = [self.pending.popleft() for _ in range(n)]
            slot.launch(reqs)
            self.stats["batches"] += 1
            busy = sum(s.busy for s in self.slots)
            self.stats["max_busy_slots"] = max(self.stats["max_busy_slots"], busy)

    def _loop(self):
        with self.cond:
            while True:
                self._dispatch()
                if self.stop and not self.pending and not any(s.busy for s in self.slots):
                    return
                self.cond.wait()

    def close(self):
        with self.cond:
            self.stop = True
            self.cond.notify_all()
        self.thread.join()
        for s in list(self.slots):
            s.close()
        self.slots = []


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
