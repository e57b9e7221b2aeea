"""Host-side scheduling logic of the server (CPU only): batch forming, slot
class choice and the arena every slot's device memory is carved from."""
import random

from paper_1604_01879_amd.sched import ALIGN, Arena, form_batch, pick_class


def test_form_batch_respects_queries_and_views():
    assert form_batch([10, 20, 30], 8, 64) == 3
    assert form_batch([10, 20, 30, 10], 8, 60) == 3
    assert form_batch([40, 40], 8, 64) == 1          # second would overflow the views
    assert form_batch([5] * 20, 8, 1000) == 8        # query slots
    assert form_batch([70, 1], 8, 64) == 0           # head too large: nothing admitted
    assert form_batch([], 8, 64) == 0


def test_form_batch_keeps_arrival_order():
    # a later small request is not admitted ahead of an earlier large one
    assert form_batch([30, 40, 1], 8, 64) == 1


def test_pick_class_smallest_that_holds_the_batch():
    classes = [(1, 64), (4, 256), (16, 1024), (64, 4096)]
    assert pick_class(1, 64, classes) == 0
    assert pick_class(1, 65, classes) == 1          # views decide: the 4-query class
    assert pick_class(2, 40, classes) == 1
    assert pick_class(5, 100, classes) == 2
    assert pick_class(64, 4096, classes) == 3
    assert pick_class(65, 10, classes) is None


def test_arena_first_fit_alignment_and_merge():
    a = Arena(10 * ALIGN)
    x = a.alloc(1)
    y = a.alloc(ALIGN + 1)
    z = a.alloc(3 * ALIGN)
    assert (x, y, z) == (0, ALIGN, 3 * ALIGN)
    assert a.alloc(5 * ALIGN) is None        # only 4 * ALIGN left
    assert a.in_use() == 6 * ALIGN
    a.release(y)
    assert a.alloc(2 * ALIGN) == ALIGN       # first fit reuses the hole
    a.release(x)
    a.release(z)
    a.release(ALIGN)
    assert a.free == [(0, 10 * ALIGN)] and a.in_use() == 0


def test_arena_random_workload_never_overlaps():
    rng = random.Random(3)
    a = Arena(64 * ALIGN)
    live = {}
    for _ in range(2000):
        if live and rng.random() < 0.45:
            off = rng.choice(list(live))
            a.release(off)
            del live[off]
        else:
            n = rng.randint(1, 12 * ALIGN)
            off = a.alloc(n)
            if off is not None:
                assert off % ALIGN == 0 and off + n <= a.size
                live[off] = n
        spans = sorted((o, o + (n + ALIGN - 1) // ALIGN * ALIGN) for o, n in live.items())
        assert all(e0 <= s1 for (_, e0), (s1, _) in zip(spans, spans[1:]))
        assert a.in_use() + sum(length for _, length in a.free) == a.size
