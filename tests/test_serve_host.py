"""Host-side scheduling logic of the server (CPU only)."""
from paper_1604_01879_amd.sched import form_batch, slots_for_budget


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


def test_slots_for_budget():
    assert slots_for_budget(10, None, 3) == 3
    assert slots_for_budget(10, 25, 3) == 2
    assert slots_for_budget(10, 5, 3) == 1
    assert slots_for_budget(10, 1000, 3) == 3
