"""Batch-forming and admission policy of the server (no device code)."""


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


def slots_for_budget(bytes_per_slot, budget_bytes, max_slots=4):
    """How many plan slots fit a device-memory budget (at least one)."""
    if budget_bytes is None:
        return max_slots
    return max(1, min(max_slots, int(budget_bytes // max(1, bytes_per_slot))))
