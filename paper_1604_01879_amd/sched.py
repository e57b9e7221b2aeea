"""Admission policy of the server (host bookkeeping only, no device code).

The server keeps plan slots in a few capacity classes (queries, views) and
pays for each slot's device memory (plan workspace plus its query-view
buffer) from one byte budget.  `Arena` hands out aligned byte ranges of that
budget; `form_batch` takes pending requests in arrival order; `pick_class`
sizes a slot for a batch.
"""
from __future__ import annotations

ALIGN = 256


def form_batch(pending, max_queries, max_views):
    """Number of leading pending requests admitted into one batch: in arrival
    order while the batch keeps within max_queries requests and max_views
    views.  A request larger than max_views is never admitted (returns 0 if
    it is first; the caller rejects it)."""
    n, views = 0, 0
    for m in pending:
        if n == max_queries or views + m > max_views:
            break
        n += 1
        views += m
    return n


def pick_class(n_queries, n_views, classes):
    """Index of the smallest capacity class (max_queries, max_views) that
    holds a batch of n_queries requests and n_views views, or None."""
    best = None
    for i, (q, v) in enumerate(classes):
        if n_queries <= q and n_views <= v and (best is None or (q, v) < classes[best]):
            best = i
    return best


class Arena:
    """First-fit allocation of ALIGN-aligned byte ranges of [0, size), with
    adjacent free ranges merged on release.  Bookkeeping only: the caller
    maps offsets into its own device buffer."""

    def __init__(self, size):
        self.size = int(size)
        self.free = [(0, self.size)]  # (offset, length), sorted, disjoint
        self.used = {}

    def alloc(self, nbytes):
        n = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        for i, (off, length) in enumerate(self.free):
            if length >= n:
                if length == n:
                    del self.free[i]
                else:
                    self.free[i] = (off + n, length - n)
                self.used[off] = n
                return off
        return None

    def release(self, off):
        n = self.used.pop(off)
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, length in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + length)
            else:
                merged.append((o, length))
        self.free = merged

    def largest_free(self):
        return max((length for _, length in self.free), default=0)

    def in_use(self):
        return sum(self.used.values())
