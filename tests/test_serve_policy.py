"""Admission order of the serving loop (host logic only, no GPU): which arrived request is
admitted next under each policy, given free memory and slots."""
import pytest

from paper_1410_4194_amd import serve as S


def _reqs(spec):
    """spec: (arrival, cost, bytes) per request, already in arrival order."""
    reqs = [S.Request(i, a, None, 1.0, cost=c) for i, (a, c, _) in enumerate(spec)]
    need = {i: b for i, (_, _, b) in enumerate(spec)}
    return reqs, (lambda r: need[r.rid])


SPEC = [(0.0, 50.0, 8), (0.1, 5.0, 2), (0.2, 1.0, 4), (5.0, 0.5, 1)]


def test_fifo_takes_the_earliest_arrival_and_stops_when_it_does_not_fit():
    reqs, need = _reqs(SPEC)
    assert S.next_admission(reqs, 1.0, 10, 4, need, "fifo") == 0
    # the head needs 8 bytes: nothing overtakes it
    assert S.next_admission(reqs, 1.0, 7, 4, need, "fifo") is None
    assert S.next_admission(reqs[1:], 1.0, 7, 4, need, "fifo") == 0


def test_sjf_takes_the_least_work_that_fits_among_arrivals():
    reqs, need = _reqs(SPEC)
    # request 3 (least cost) has not arrived at t = 1
    assert S.next_admission(reqs, 1.0, 10, 4, need, "sjf") == 2
    # request 2 (4 bytes) does not fit in 3: request 1 (cost 5, 2 bytes) does
    assert S.next_admission(reqs, 1.0, 3, 4, need, "sjf") == 1
    assert S.next_admission(reqs, 6.0, 10, 4, need, "sjf") == 3
    assert S.next_admission(reqs, 1.0, 1, 4, need, "sjf") is None


def test_sjf_breaks_ties_by_arrival():
    reqs, need = _reqs([(0.0, 2.0, 1), (0.1, 1.0, 1), (0.2, 1.0, 1)])
    assert S.next_admission(reqs, 1.0, 10, 4, need, "sjf") == 1


@pytest.mark.parametrize("policy", S.POLICIES)
def test_no_free_slot_admits_nothing(policy):
    reqs, need = _reqs(SPEC)
    assert S.next_admission(reqs, 1.0, 100, 0, need, policy) is None
    assert S.next_admission([], 1.0, 100, 4, need, policy) is None


def test_unknown_policy_is_refused():
    reqs, need = _reqs(SPEC)
    with pytest.raises(ValueError):
        S.next_admission(reqs, 1.0, 100, 4, need, "lifo")
