"""CPU checks of the binomial checkpointing schedule (sps_checkpoint_schedule, host code; no
device): every action is executable (each advance starts where the working state is, each
load finds the state it names in its slot, each turn finds X_i in hand, at most `slots` states
are stored at once), the reverse sweep turns every step exactly once in the order N-1 .. 0, and
the number of forward steps equals the minimum over all schedules, computed here by brute-force
dynamic programming over every split and checked against the closed form
r n - C(c + r, r - 1) (c stored states, r the smallest pass count with C(c + r, c) >= n).
The schedule with priced stores and loads (sps_checkpoint_schedule_costs) is checked the same
way, its reported cost against the cost of its actions and against an exhaustive search over
every schedule on small runs."""
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


# ---------------------------------------------------------------------------- schedules with costs
# (sps_checkpoint_schedule_costs: a forward step of the reverse sweep costs adv, storing a state
# wr, loading one rd; the outer level of the nested two-level schedule)

def priced(fwd, rev, n, slots, adv, wr, rd):
    """The cost of a schedule counted from its actions (after checking that it is executable)."""
    _, adv_r, _ = simulate(fwd, rev, n, slots)
    shots = sum(1 for op, _, _ in fwd + rev if op == TAKESHOT)
    loads = sum(1 for op, _, _ in rev if op == RESTORE)
    return adv * adv_r + wr * shots + rd * loads


def exhaustive_min_cost(n, slots, adv, wr, rd):
    """Least cost over every schedule with at most `slots` stored states (shortest path over
    states: phase, working state, stored set, steps left to reverse).  The forward sweep runs
    0 -> n at no cost and may store states on the way (X_0 always); in the reverse sweep a
    stored state may be dropped at no cost, loaded (rd), the working state advanced one step
    (adv) or stored (wr), and step k - 1 reversed when the working state holds X_{k-1}; after a
    reversal the working state is spent."""
    import heapq
    start = ("f", 0, frozenset([0]), n)
    dist = {start: wr}
    heap = [(wr, 0, start)]
    tick = 1
    while heap:
        c, _, st = heapq.heappop(heap)
        if dist.get(st, float("inf")) < c - 1e-12:
            continue
        ph, w, S, k = st
        if ph == "r" and k == 0:
            return c
        moves = []
        if ph == "f":
            if w < n:
                moves.append((0.0, ("f", w + 1, S, k)))
                if w not in S and len(S) < slots:
                    moves.append((wr, ("f", w, S | {w}, k)))
            else:
                moves.append((0.0, ("r", n, S, n)))
        else:
            for p in S:
                if p != 0:
                    moves.append((0.0, ("r", w, S - {p}, k)))
                if p < k and p != w:
                    moves.append((rd, ("r", p, S, k)))
            if w < k - 1:
                moves.append((adv, ("r", w + 1, S, k)))
                if w not in S and len(S) < slots:
                    moves.append((wr, ("r", w, S | {w}, k)))
            if w == k - 1:
                kept = frozenset(p for p in S if p < k - 1) | ({0} if k > 1 else frozenset())
                moves.append((0.0, ("r", k, kept if k > 1 else frozenset(), k - 1)))
        for dc, nxt in moves:
            if c + dc < dist.get(nxt, float("inf")) - 1e-12:
                dist[nxt] = c + dc
                heapq.heappush(heap, (c + dc, tick, nxt))
                tick += 1
    raise AssertionError("no schedule")


COSTS = [(1.0, 0.0, 0.0), (1.0, 0.5, 0.5), (1.0, 2.0, 0.0), (1.0, 0.0, 2.0), (1.0, 3.0, 1.0), (2.0, 1.0, 5.0),
         (1.0, 10.0, 10.0), (1.0, 0.3, 4.0)]


@pytest.mark.parametrize("costs", COSTS)
def test_cost_schedule_is_the_least_cost_schedule(costs):
    """On runs of up to 7 steps with 1-3 slots the schedule is executable, the cost it reports is
    the cost of its actions, and no schedule at all costs less (exhaustive search)."""
    adv, wr, rd = costs
    for n in range(1, 8):
        for slots in range(1, 4):
            fwd, rev, c = sps.checkpoint_schedule_costs(n, slots, adv, wr, rd)
            assert abs(priced(fwd, rev, n, slots, adv, wr, rd) - c) < 1e-9, (n, slots)
            assert abs(exhaustive_min_cost(n, slots, adv, wr, rd) - c) < 1e-9, (n, slots)


@pytest.mark.parametrize("n,slots", [(10, 3), (50, 4), (137, 5), (20, 20)])
def test_cost_schedule_without_costs_needs_the_fewest_steps(n, slots):
    """With free stores and loads the schedule recomputes as few steps as the binomial one."""
    fwd, rev, c = sps.checkpoint_schedule_costs(n, slots, 1.0, 0.0, 0.0)
    _, adv_r, _ = simulate(fwd, rev, n, slots)
    _, adv_b, _ = simulate(*sps.checkpoint_schedule(n, slots), n, slots)
    assert adv_r == adv_b == c


def test_cost_schedule_trades_steps_for_stores():
    """Dear stores: fewer states stored and more steps recomputed; a store dearer than all the
    recomputation it can save: none besides X_0."""
    n, slots = 40, 6
    counts = []
    for wr in (0.0, 2.0, 8.0, 1e6):
        fwd, rev, c = sps.checkpoint_schedule_costs(n, slots, 1.0, wr, 0.5)
        _, adv_r, _ = simulate(fwd, rev, n, slots)
        counts.append((sum(1 for op, _, _ in fwd + rev if op == TAKESHOT), adv_r))
    shots, steps = zip(*counts)
    assert list(shots) == sorted(shots, reverse=True) and list(steps) == sorted(steps)
    assert shots[-1] == 1 and steps[-1] == n * (n - 1) // 2


def test_cost_schedule_bad_arguments():
    for args in ((0, 3, 1.0, 0.0, 0.0), (10, 0, 1.0, 0.0, 0.0), (10, 3, -1.0, 0.0, 0.0), (10, 3, 1.0, float("nan"), 0.0),
                 (100000, 1000, 1.0, 1.0, 1.0)):   # (the last: more work than the search accepts)
        with pytest.raises(sps.SpsError):
            sps.checkpoint_schedule_costs(*args)
