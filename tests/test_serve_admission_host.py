"""Host logic of the server's admission: a request larger than the whole
memory budget is refused, others wait for a free slot and for memory, and
released memory and slots are reused.  Pure host code: no GPU."""
from paper_2507_04775_amd.serve import Admission


def test_oversized_request_is_refused_even_when_idle():
    a = Admission(slots=4, budget=100)
    assert a.refuses(101)
    assert not a.refuses(100)
    assert a.admit(100) is not None


def test_admission_waits_for_memory_and_slots_then_reuses_them():
    a = Admission(slots=2, budget=100)
    s0 = a.admit(60)
    assert s0 is not None
    assert a.admit(50) is None          # memory: 60 + 50 > 100
    s1 = a.admit(40)
    assert s1 is not None and s1 != s0
    assert a.admit(1) is None           # no slot left
    a.release(s0, 60)
    assert a.used == 40
    s2 = a.admit(50)
    assert s2 == s0
    assert a.used == 90
    a.release(s1, 40)
    a.release(s2, 50)
    assert a.used == 0 and sorted(a.free) == [0, 1]
