"""CPU checks of the binomial checkpointing schedule (sps_checkpoint_schedule, host code; no
device): every action is executable (each advance starts where the working state is, each
load finds the state it names in its slot, each turn finds X_i in hand, at most `slots` states
are stored at once), the reverse sweep turns every step exactly once in the order N-1 .. 0, and
the number of forward steps equals the minimum over all schedules, computed here by brute-force
dynamic programming over every split and checked against the closed form
r n - C(c + r, r - 1) (c stored states, r the smallest pass count with C(c + r, c) >= n)."""
from functools import lru_cache
from math import comb

import pytest

import paper_2506_14792_amd as sps

ADVANCE, TAKESHOT, RESTORE, YOUTURN = 1, 2, 3, 4


@lru_cache(None)
def min_advances(n, s):
    """Fewest unrecorded forward steps to reverse n steps whose first state is stored, with s
    more free slots: try every first snapshot position m (brute force)."""
    if n == 1:
        return 0
    if s == 0:
        return n * (n - 1) // 2          # restart from the stored state for every step
    return min(m + min_advances(n - m, s - 1) + min_advances(m, s) for m in range(1, n))


def closed_form(n, c):
    r = 0
    while comb(c + r, c) < n:
        r += 1
    return r * n - (comb(c + r, r - 1) if r >= 1 else 0)


def simulate(fwd, rev, n, slots):
    snaps, w, adv_f, adv_r, turns = {}, 0, 0, 0, []
    last_shot = 0
    for op, a, b in fwd:
        if op == TAKESHOT:
            assert w == b and 0 <= a < slots
            snaps[a] = b
            last_shot = b
        elif op == ADVANCE:
            assert w == a and a < b <= n
            adv_f += b - a
            w = b
        else:
            raise AssertionError(f"forward sweep action {op}")
    assert w == n
    for op, a, b in rev:
        if op == RESTORE:
            assert snaps.get(a) == b
            w = b
        elif op == TAKESHOT:
            assert w == b and 0 <= a < slots
            snaps[a] = b
        elif op == ADVANCE:
            assert w == a and a < b < n
            adv_r += b - a
            w = b
        elif op == YOUTURN:
            assert w == a
            turns.append(a)
            w = a + 1
        else:
            raise AssertionError(op)
    assert turns == list(range(n - 1, -1, -1))
    return adv_f, adv_r, last_shot


def test_brute_force_minimum_matches_closed_form():
    for s in range(0, 7):
        for n in range(1, 90):
            assert min_advances(n, s) == closed_form(n, s + 1), (n, s)


@pytest.mark.parametrize("slots", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("n", [1, 2, 3, 7, 10, 50, 137])
def test_schedule_is_valid_and_optimal(n, slots):
    fwd, rev = sps.checkpoint_schedule(n, slots)
    adv_f, adv_r, last_shot = simulate(fwd, rev, n, slots)
    assert adv_f == n
    # the forward sweep's advances up to its last snapshot are the first descent of an
    # optimal schedule; the reverse sweep does the rest of it
    assert adv_r == min_advances(n, slots - 1) - last_shot, (adv_r, min_advances(n, slots - 1), last_shot)


def test_enough_slots_means_no_recomputation():
    n = 40
    fwd, rev = sps.checkpoint_schedule(n, n)
    adv_f, adv_r, _ = simulate(fwd, rev, n, n)
    assert adv_f == n and adv_r == 0


def test_one_slot_recomputes_from_the_start():
    n = 12
    _, rev = sps.checkpoint_schedule(n, 1)
    _, adv_r, _ = simulate(*sps.checkpoint_schedule(n, 1), n, 1)
    assert adv_r == n * (n - 1) // 2
    assert sum(1 for op, _, _ in rev if op == RESTORE) == n


def test_bad_arguments():
    with pytest.raises(sps.SpsError):
        sps.checkpoint_schedule(0, 3)
    with pytest.raises(sps.SpsError):
        sps.checkpoint_schedule(10, 0)
