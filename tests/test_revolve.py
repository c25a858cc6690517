"""CPU checks of the binomial checkpoint schedule exported by the library
(host code, no GPU): optimal forward-step count, and a replay of the actions
that verifies every adjoint step sees the right state with at most the given
number of slots."""
import functools
from math import comb

import pytest

from paper_2302_05164_amd import pbftherm as P


def closed_form(l, c):
    """r l - C(c + r, r - 1), r the smallest repetition number with C(c + r, c) >= l
    (Griewank's binomial checkpointing)."""
    r = 0
    while comb(c + r, c) < l:
        r += 1
    return r * l - (comb(c + r, r - 1) if r >= 1 else 0)


@functools.lru_cache(maxsize=None)
def brute_force(l, c):
    """Fewest forward steps to reverse l steps holding at most c states (the
    initial one included): either step the initial state forward each time
    (c == 1), or advance m steps, store, reverse the right part with c - 1
    slots and the left part with c."""
    if l == 1:
        return 0
    if c == 1:
        return l * (l - 1) // 2
    return min(m + brute_force(l - m, c - 1) + brute_force(m, c) for m in range(1, l))


def replay(acts, l, c):
    """Execute the actions symbolically; returns (turn order, advances)."""
    slots = {}
    cur = 0
    turns, adv = [], 0
    for kind, step, slot in acts:
        if kind == P.ACT_ADVANCE:
            assert step > cur
            adv += step - cur
            cur = step
        elif kind == P.ACT_STORE:
            assert step == cur and 0 <= slot < c
            slots[slot] = cur
        elif kind == P.ACT_RESTORE:
            assert slots.get(slot) == step
            cur = step
        elif kind == P.ACT_TURN:
            assert step == cur
            turns.append(step)
        else:
            raise AssertionError(kind)
    return turns, adv


def test_forward_step_count_is_minimal():
    for c in range(1, 7):
        for l in range(1, 70):
            _, adv = P.revolve_schedule(l, c, with_actions=False)
            assert adv == closed_form(l, c) == brute_force(l, c), (l, c)


@pytest.mark.parametrize("l,c", [(1, 1), (2, 1), (7, 1), (10, 3), (37, 4), (100, 5), (200, 200),
                                 (3000, 30)])
def test_replay_turns_every_step_once_in_reverse(l, c):
    acts, adv = P.revolve_schedule(l, c)
    assert acts[0] == (P.ACT_STORE, 0, 0)
    turns, adv2 = replay(acts, l, c)
    assert turns == list(range(l - 1, -1, -1))
    assert adv2 == adv == closed_form(l, c)


def test_three_thousand_steps_thirty_slots():
    # r = 3: C(33, 3) = 5456 >= 3000 > C(32, 2) = 496; 3 * 3000 - C(33, 2) = 8472
    assert P.revolve_schedule(3000, 30, with_actions=False)[1] == 8472


def test_enough_slots_means_one_sweep():
    for l in (1, 2, 5, 64):
        assert P.revolve_schedule(l, l, with_actions=False)[1] == l - 1
        assert P.revolve_schedule(l, 10 * l, with_actions=False)[1] == l - 1


def test_invalid_requests():
    with pytest.raises(P.PbfError):
        P.revolve_schedule(0, 4)
    with pytest.raises(P.PbfError):
        P.revolve_schedule(10, 0)
