"""Host-side model of the persistent batch kernel's work queue.

The persistent F-IF batch kernel numbers its work items phase by phase (split
and quantize, codeword dots, clear, word selection, word offsets, grouping,
active tiles, list scan, per-query mean) and lets blocks take them in
increasing order from one counter; the clear of the match buffer has no
items of its own but runs inside the dot-tile items.  An item waits until a
`done` counter reaches the first item number of its phase (the dot tiles
wait on a counter of finished split items instead), and the first
item at or past the list scan waits for every item before the scan and then
learns how many scan items there are.  Each block takes one acquire per phase
after its wait; producers release before they count themselves done.

This model re-derives the item ranges from the same formulas and runs the
queue under many random schedules (random block counts, item durations and
interleavings).  For every schedule it checks what the kernel's correctness
rests on:

* the queue drains (no schedule deadlocks);
* every query view is split and quantized by exactly one item, and every
  word of the match buffer rows [0, n_v) is cleared by exactly one item;
* every item starts only after every item that produces its inputs has
  finished, and its block took an acquire after those items finished;
* every clear of a match-buffer row finishes before any list-scan item that
  writes to that row starts, and every list-scan item finishes before any
  per-query-mean item that reads its (view, shape) entries starts;
* every score S[b][p] of the batch (b < n_q, p < N) is written by exactly
  one per-query-mean item.

It runs for split items of 4 views (the kernel's) and of 16 views.
"""
import numpy as np
import pytest

# phases, in item order (the kernel's BatchPhase)
Q, GEMM, FILL, SEL, PRE, SCAT, TILE, SCAN, RED = range(9)
RED_SHAPES = 4096         # shapes of one query per mean item
SEL_SPLIT_MAX = 512       # batches up to this many views: one selection item per view
LIST_TILE = 128           # list entries per scan tile


class Batch:
    """A random ragged batch and index, with the item ranges of the kernel."""

    def __init__(self, rng, n_q, n_shapes, K, q_views_per_item, big=False):
        m = rng.integers(1, 65, size=n_q)
        self.qoff = np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
        self.n_q, self.n_v, self.N, self.K = n_q, int(self.qoff[-1]), n_shapes, K
        self.qv = q_views_per_item
        # list lengths and each query view's word
        lens = rng.integers(0, 3 * LIST_TILE, size=K)
        if big:
            lens[rng.integers(0, K)] = 40 * LIST_TILE
        self.tiles_of = [(int(l) + LIST_TILE - 1) // LIST_TILE for l in lens]
        self.words = rng.integers(0, K, size=self.n_v)
        # a list tile's entries: random shapes (only which shapes matter here)
        self.tile_shapes = [[rng.integers(0, n_shapes, size=min(LIST_TILE, int(lens[w]) - t *
                                                                 LIST_TILE))
                             for t in range(self.tiles_of[w])] for w in range(K)]
        gemm_col_tiles = (K + 127) // 128
        n_items = [
            (self.n_v + self.qv - 1) // self.qv,
            ((self.n_v + 127) // 128) * gemm_col_tiles,
            0,  # the clear runs inside the GEMM items
            self.n_v if self.n_v <= SEL_SPLIT_MAX else (self.n_v + 3) // 4,
            1,
            (self.n_v + 255) // 256,
            (K + 255) // 256,
        ]
        self.first = np.concatenate([[0], np.cumsum(n_items)]).astype(np.int64)
        # what PRE computes: tiles of the lists that have query views, in word order
        used = np.zeros(K, bool)
        used[self.words] = True
        self.act = [(w, t) for w in range(K) if used[w] for t in range(self.tiles_of[w])]
        self.n_active = len(self.act)
        self.red_chunks = (n_shapes + RED_SHAPES - 1) // RED_SHAPES
        self.n_red = n_q * self.red_chunks
        self.group = {w: np.nonzero(self.words == w)[0] for w in range(K) if used[w]}

    def phase_of(self, item):
        """(phase, index in phase, `done` value the item waits for or None)."""
        if item < self.first[SCAN]:
            ph = int(np.searchsorted(self.first, item, side="right") - 1)
            return ph, item - int(self.first[ph]), int(self.first[ph])
        j = item - int(self.first[SCAN])
        if j < self.n_active:
            return SCAN, j, None
        j -= self.n_active
        if j < self.n_red:
            return RED, j, int(self.first[SCAN]) + self.n_active
        return None, None, None


def simulate(b: Batch, n_blocks: int, rng):
    """Runs the queue with n_blocks blocks under a random interleaving.

    Returns the event log: per item (block, phase, j, start, end, acquire
    time that covered it)."""
    head = done = q_done = 0
    t = 0
    # per block: state, current item, remaining work, acquired phase, last
    # acquire time, whether it knows n_active
    blocks = [dict(state="take", acq=-1, acq_t=-1, knows_active=False, item=None, left=0,
                   ph=None, j=None, need=None) for _ in range(n_blocks)]
    log = {}
    finished = 0
    while True:
        runnable = [i for i, s in enumerate(blocks) if s["state"] != "exit"]
        if not runnable:
            break
        progressed = False
        for bi in rng.permutation(runnable):
            s = blocks[bi]
            t += 1
            if s["state"] == "take":
                s["item"] = head
                head += 1
                s["state"] = "classify"
                progressed = True
                break
            if s["state"] == "classify":
                item = s["item"]
                if item >= b.first[SCAN] and not s["knows_active"]:
                    # thread 0 waits for every item before the scan, acquires,
                    # then reads the number of active tiles PRE published
                    if done < b.first[SCAN]:
                        continue
                    s["knows_active"] = True
                    s["acq"], s["acq_t"] = SCAN, t
                ph, j, need = b.phase_of(item)
                if ph is None:
                    s["state"] = "exit"
                    progressed = True
                    break
                s["ph"], s["j"], s["need"] = ph, j, need
                s["state"] = "wait"
                progressed = True
                break
            if s["state"] == "wait":
                ph = s["ph"]
                needs_wait = ph in (GEMM, SEL, PRE, SCAT, TILE, RED)
                if needs_wait and ph > s["acq"]:
                    if ph == GEMM:
                        if q_done < b.first[GEMM]:
                            continue
                    elif done < s["need"]:
                        continue
                    s["acq"], s["acq_t"] = ph, t
                s["state"] = "run"
                s["start"] = t
                s["left"] = int(rng.integers(1, 6))
                progressed = True
                break
            if s["state"] == "run":
                s["left"] -= 1
                if s["left"] == 0:
                    log[s["item"]] = dict(block=bi, ph=s["ph"], j=s["j"], start=s["start"],
                                          end=t, acq_t=s["acq_t"])
                    if s["ph"] == Q:
                        q_done += 1
                    if s["ph"] != RED:
                        done += 1
                    finished += 1
                    s["state"] = "take"
                progressed = True
                break
        assert progressed, f"deadlock: head={head} done={done} q_done={q_done}"
    return log


def check(b: Batch, log):
    by_ph = {}
    for it, e in log.items():
        by_ph.setdefault(e["ph"], []).append((it, e))
    n_items = int(b.first[SCAN]) + b.n_active + b.n_red
    assert sorted(log) == list(range(n_items)), "every item runs exactly once"

    def end_of(ph):
        return max((e["end"] for _, e in by_ph.get(ph, [])), default=-1)

    # split / quantize covers every view once
    cover = np.zeros(b.n_v, int)
    for _, e in by_ph.get(Q, []):
        for v in range(e["j"] * b.qv, min(e["j"] * b.qv + b.qv, b.n_v)):
            cover[v] += 1
    assert (cover == 1).all()
    # the clear (a share of it in every GEMM item) covers every word of rows
    # [0, n_v) once
    words = b.n_v * b.N
    n_gemm = int(b.first[FILL] - b.first[GEMM])
    per = ((words + n_gemm - 1) // n_gemm + 1023) // 1024 * 1024
    assert not by_ph.get(FILL)
    fill_cover = np.zeros(words, np.int8)
    fill_end = np.full(words, -1.0)
    for _, e in by_ph.get(GEMM, []):
        e0, e1 = e["j"] * per, min(e["j"] * per + per, words)
        fill_cover[e0:e1] += 1
        fill_end[e0:e1] = e["end"]
    assert (fill_cover == 1).all()
    # producers finish before consumers start, and the consumer's block
    # acquired after they finished
    producers = {GEMM: [Q], SEL: [Q, GEMM, FILL], PRE: [Q, GEMM, FILL, SEL],
                 SCAT: [Q, GEMM, FILL, SEL, PRE], TILE: [Q, GEMM, FILL, SEL, PRE, SCAT],
                 SCAN: [Q, GEMM, FILL, SEL, PRE, SCAT, TILE],
                 RED: [Q, GEMM, FILL, SEL, PRE, SCAT, TILE, SCAN]}
    for ph, prods in producers.items():
        last = max(end_of(p) for p in prods)
        for it, e in by_ph.get(ph, []):
            assert e["start"] > last, (ph, it)
            assert e["acq_t"] > last, (ph, it, "acquire before the producers finished")
    # clear of a row before any scan of that row; scans of (view, shape) before
    # the mean that reads them
    scan_end = {}
    for _, e in by_ph.get(SCAN, []):
        w, tt = b.act[e["j"]]
        for v in b.group[w]:
            w0, w1 = v * b.N, (v + 1) * b.N - 1
            assert e["start"] > fill_end[w0:w1 + 1].max()
            row = scan_end.setdefault(int(v), {})
            for p in b.tile_shapes[w][tt]:
                row[int(p)] = max(row.get(int(p), -1), e["end"])
    s_written = np.zeros((b.n_q, b.N), int)
    for _, e in by_ph.get(RED, []):
        q = e["j"] // b.red_chunks
        p0 = (e["j"] - q * b.red_chunks) * RED_SHAPES
        p1 = min(b.N, p0 + RED_SHAPES)
        s_written[q, p0:p1] += 1
        for v in range(int(b.qoff[q]), int(b.qoff[q + 1])):
            for p, t_end in scan_end.get(v, {}).items():
                if p0 <= p < p1:
                    assert e["start"] > t_end
    assert (s_written == 1).all(), "every batch score written exactly once"


@pytest.mark.parametrize("q_views_per_item", [4, 16])
@pytest.mark.parametrize("seed", range(6))
def test_queue_schedules(q_views_per_item, seed):
    rng = np.random.default_rng(1000 + seed)
    b = Batch(rng, n_q=int(rng.integers(1, 10)), n_shapes=int(rng.integers(200, 2600)),
              K=int(rng.integers(20, 300)), q_views_per_item=q_views_per_item, big=seed % 2 == 1)
    for n_blocks in (1, 2, 7, 32):
        check(b, simulate(b, n_blocks, rng))


def test_queue_model_detects_a_missing_wait():
    """The checker itself: a queue whose per-query means skip their wait
    must be caught under some schedule."""
    rng = np.random.default_rng(7)
    b = Batch(rng, n_q=4, n_shapes=700, K=40, q_views_per_item=4)
    b.phase_of_orig = b.phase_of

    def no_red_wait(item):
        ph, j, need = b.phase_of_orig(item)
        return (ph, j, 0) if ph == RED else (ph, j, need)

    b.phase_of = no_red_wait
    caught = False
    for _ in range(20):
        try:
            check(b, simulate(b, 16, rng))
        except AssertionError:
            caught = True
            break
    assert caught
