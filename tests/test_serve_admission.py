"""Admission logic of the serving loop (host only, no GPU)."""
import pytest

from paper_1405_2255_amd.serve import Admission


def test_fifo_slots_and_bytes():
    a = Admission(slots=2, budget_bytes=100)
    assert a.push("r1", 60) and a.push("r2", 30) and a.push("r3", 50)
    assert a.pop_admissible() == ("r1", 60, 0, [])
    assert a.pop_admissible() == ("r2", 30, 1, [])
    # both slots busy
    assert a.pop_admissible() is None
    a.release(1)
    # a slot is free, but slot 1 growing to 50 next to slot 0's 60 exceeds 100
    assert a.pop_admissible() is None
    a.release(0)
    # slot 0 already holds 60 >= 50: no growth
    assert a.pop_admissible() == ("r3", 50, 0, [])
    assert a.running == 1 and a.used == 90


def test_head_of_line_order_is_kept():
    a = Admission(slots=4, budget_bytes=100)
    a.push("big", 90)
    a.push("small", 5)
    assert a.pop_admissible() == ("big", 90, 0, [])
    # small fits, and is next in line
    assert a.pop_admissible() == ("small", 5, 1, [])


def test_idle_slots_keep_their_bytes():
    # a context keeps its largest buffers: an idle slot still counts
    a = Admission(slots=2, budget_bytes=100)
    a.push("r1", 70)
    assert a.pop_admissible() == ("r1", 70, 0, [])
    a.release(0)
    a.push("r2", 20)
    # slot 0 is free and already holds 70: r2 runs there without growth
    assert a.pop_admissible() == ("r2", 20, 0, [])
    a.push("r3", 25)
    # slot 1 would hold 25 next to slot 0's 70: fits
    assert a.pop_admissible() == ("r3", 25, 1, [])
    assert a.used == 95


def test_idle_slot_emptied_when_needed():
    a = Admission(slots=3, budget_bytes=100)
    for name, nb in (("a", 40), ("b", 40), ("c", 10)):
        a.push(name, nb)
    assert [a.pop_admissible()[2] for _ in range(3)] == [0, 1, 2]
    for s in (0, 1, 2):
        a.release(s)
    # 70 grows one slot; the held bytes of the others must go first: slot 0 runs
    # it (ties to the lower slot) and the largest idle slot (1) is emptied
    a.push("d", 70)
    item, nb, slot, empty = a.pop_admissible()
    assert (item, slot, empty) == ("d", 0, [1])
    assert a.held == [70, 0, 10] and a.used == 80
    # a running slot is never emptied: 95 cannot start until slot 0 is free
    a.push("e", 95)
    assert a.pop_admissible() is None
    a.release(0)
    item, nb, slot, empty = a.pop_admissible()
    assert (item, slot, empty) == ("e", 0, [2])
    assert a.used == 95 <= a.budget


def test_oversized_request_refused():
    a = Admission(slots=1, budget_bytes=10)
    assert not a.push("huge", 11)
    assert a.pop_admissible() is None


def test_bad_configuration():
    with pytest.raises(ValueError):
        Admission(slots=0, budget_bytes=10)
    with pytest.raises(ValueError):
        Admission(slots=1, budget_bytes=0)
