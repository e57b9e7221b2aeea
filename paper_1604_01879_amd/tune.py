"""Autotuner of batch plans.

A plan's persistent first-pass kernel has three settings that change its
speed but not its ranked ids: the persistent blocks per CU, the number of
list entries one scan item covers (list tile), and the largest query-view
group that takes the narrow scan tile.  `tune_plan` times every candidate
setting on a representative batch of a plan configuration (database size,
storage, vocabulary, capacities) and keeps the fastest; the choice and the
timing grid are cached as JSON, keyed by the configuration, so later plans
of the same configuration start tuned.

Only the timing loop lives here; every run is a libgift plan.
"""
from __future__ import annotations

import json
import os
import tempfile

import torch

from . import _lib as L

CANDIDATES = [dict(blocks_per_cu=b, list_tile=t, narrow_max=n)
              for b in (1, 2) for t in (64, 128) for n in (0, 16, 32)]
DEFAULT = dict(blocks_per_cu=2, list_tile=128, narrow_max=32)


def default_cache_path():
    return os.environ.get("GIFT_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "gift", "plan_tuning.json")


def config_key(db: L.Views, fif: L.Fif, max_queries, max_views, max_m, top_k, rescore_r):
    """The plan configuration a tuning applies to."""
    return (f"N{db.n_shapes}-v{db.n_views}-d{db.dim}-dt{db.dtype}-K{fif.K}-ma{fif.ma}"
            f"-q{max_queries}-V{max_views}-m{max_m}-k{top_k}-r{rescore_r}")


def load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(path, cache):
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_plan(plan: L.FifPlan, n_queries, n_views, reps):
    """Average ms per run of a loaded plan (events on its stream)."""
    plan.run(n_queries, n_views)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(plan.stream)
    for _ in range(reps):
        plan.run(n_queries, n_views)
    e1.record(plan.stream)
    plan.stream.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_plan(db: L.Views, fif: L.Fif, q_views, q_offsets, max_m, top_k, rescore_r,
              max_queries=None, max_views=None, candidates=None, reps=3, cache_path=None,
              refresh=False):
    """The fastest candidate setting for plans of this configuration on the
    batch (q_views float32 device [n_v, dim], q_offsets int [n_q + 1]):
    returns (setting dict, cache entry).  A cached entry is returned without
    timing unless `refresh`."""
    offsets = torch.as_tensor(q_offsets, dtype=torch.int32).cpu()
    n_q, n_v = int(offsets.numel() - 1), int(offsets[-1])
    max_queries = max_queries or n_q
    max_views = max_views or n_v
    path = cache_path or default_cache_path()
    key = config_key(db, fif, max_queries, max_views, max_m, top_k, rescore_r)
    cache = load_cache(path)
    if key in cache and not refresh:
        return dict(cache[key]["best"]), cache[key]
    grid = []
    for cand in candidates or CANDIDATES:
        plan = L.FifPlan(db, fif, max_queries, max_views, max_m, top_k, rescore_r, **cand)
        try:
            plan.views[:n_v].copy_(q_views[:n_v])
            plan.offsets[:n_q + 1].copy_(offsets.to(plan.offsets.device))
            torch.cuda.synchronize()
            ms = time_plan(plan, n_q, n_v, reps)
            grid.append(dict(cand, ms=round(ms, 4), queue_error=plan.error()))
        finally:
            plan.close()
    ok = [g for g in grid if g["queue_error"] == 0]
    best = min(ok or grid, key=lambda g: g["ms"])
    entry = {"best": {k: best[k] for k in DEFAULT}, "ms_grid": grid,
             "batch": {"queries": n_q, "views": n_v}, "reps": reps}
    cache[key] = entry
    _save_cache(path, cache)
    return dict(entry["best"]), entry
