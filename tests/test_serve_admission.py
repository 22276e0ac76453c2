"""Admission logic of the serving loop (host only, no GPU)."""
import pytest

from paper_1405_2255_amd.serve import Admission


def test_fifo_slots_and_bytes():
    a = Admission(slots=2, budget_bytes=100)
    assert a.push("r1", 60) and a.push("r2", 30) and a.push("r3", 50)
    assert a.pop_admissible() == ("r1", 60)
    assert a.pop_admissible() == ("r2", 30)
    # both slots busy
    assert a.pop_admissible() is None
    a.release(30)
    # a slot is free but r3 (50) does not fit next to r1 (60)
    assert a.pop_admissible() is None
    a.release(60)
    assert a.pop_admissible() == ("r3", 50)
    assert a.running == 1 and a.used == 50


def test_head_of_line_order_is_kept():
    a = Admission(slots=4, budget_bytes=100)
    a.push("big", 90)
    a.push("small", 5)
    assert a.pop_admissible() == ("big", 90)
    # small fits, and is next in line
    assert a.pop_admissible() == ("small", 5)


def test_oversized_request_refused():
    a = Admission(slots=1, budget_bytes=10)
    assert not a.push("huge", 11)
    assert a.pop_admissible() is None


def test_bad_configuration():
    with pytest.raises(ValueError):
        Admission(slots=0, budget_bytes=10)
    with pytest.raises(ValueError):
        Admission(slots=1, budget_bytes=0)
