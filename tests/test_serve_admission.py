"""Admission of serving requests by HBM budget (host logic, no GPU): requests
are admitted in arrival order while their device state fits beside what is
in use; a request that can never fit is rejected at once and does not block
the ones behind it."""

import collections

from paper_2602_19959_amd.serve import admit


def sizes(*xs):
    return collections.deque(xs)


def test_admits_in_order_while_it_fits():
    q = sizes(30, 30, 30, 10)
    got, rej, used = admit(q, pool_used=40, pool_bytes=120, state_room=80, size_of=lambda r: r)
    assert got == [30, 30] and rej == [] and used == 100
    assert list(q) == [30, 10]          # the head waits; nothing overtakes it


def test_request_that_can_never_fit_is_rejected_not_blocking():
    q = sizes(90, 20, 500, 20)
    got, rej, used = admit(q, pool_used=40, pool_bytes=120, state_room=80, size_of=lambda r: r)
    assert rej == [90, 500] and got == [20, 20] and used == 80 and not q


def test_exact_fit_and_empty_queue():
    got, rej, used = admit(sizes(80), pool_used=40, pool_bytes=120, state_room=80, size_of=lambda r: r)
    assert got == [80] and used == 120
    got, rej, used = admit(sizes(), pool_used=40, pool_bytes=120, state_room=80, size_of=lambda r: r)
    assert got == [] and rej == [] and used == 40


def test_full_pool_admits_nothing_but_still_rejects_oversized():
    q = sizes(200, 10)
    got, rej, used = admit(q, pool_used=120, pool_bytes=120, state_room=80, size_of=lambda r: r)
    assert rej == [200] and got == [] and list(q) == [10] and used == 120
