"""Binomial checkpoint schedules (host logic, no GPU): the number of segment
advances the library's schedule makes equals the least possible, computed
here by brute-force dynamic programming over every split, and matches
Griewank's closed form; workspace and recomputation counts follow."""
from functools import lru_cache

import pytest

import workloads as W
from paper_1504_08340_amd import binding as B


@lru_cache(maxsize=None)
def least_advances(l, s):
    """Least segment advances to reverse l segments from a held state with s
    free slots: advance m, keep, reverse the right part with s - 1 slots and
    the left part with s (brute force over m)."""
    if l <= 1:
        return 0
    if s == 0:
        return l * (l - 1) // 2
    return min(m + least_advances(l - m, s - 1) + least_advances(m, s) for m in range(1, l))


def _sizes(nsteps, k, slots, nsrc=1):
    prob = W.Problem((2, 2, 2), 1, 1, 1.0, 1e-3, nsteps)
    return B.fwi_query(B.make_problem(prob, nsrc, 1, 0, k, 0, slots))


@pytest.mark.parametrize("nseg", [2, 3, 7, 12, 25, 40])
@pytest.mark.parametrize("slots", [1, 2, 3, 5])
def test_schedule_is_optimal(nseg, slots):
    k = 3
    sz = _sizes(nseg * k, k, slots)
    if slots >= nseg - 1:
        assert sz.schedule_advances == nseg - 1 and sz.ckpt_states == nseg
    else:
        assert sz.schedule_advances == least_advances(nseg, slots)
        assert sz.ckpt_states == slots


def test_closed_form_of_the_least_advances():
    """Griewank's binomial result with S = s + 1 snapshots: t l - C(S + t, S + 1),
    t the least integer with C(S + t, S) >= l (pins the brute force)."""
    from math import comb
    for s in range(1, 6):
        for l in range(2, 60):
            S = s + 1
            t = 0
            while comb(S + t, S) < l:
                t += 1
            assert least_advances(l, s) == t * l - comb(S + t, S + 1)


def test_counts_and_memory():
    # uniform spacing: every segment start kept, each segment recomputed once
    sz = _sizes(100, 10, 0)
    assert sz.ckpt_states == 10 and sz.adjoint_forward_steps == 100
    # ragged last segment
    sz = _sizes(95, 10, 0)
    assert sz.ckpt_states == 10 and sz.adjoint_forward_steps == 95
    # three slots for 20 segments: fewer states, more recomputation
    full, rev = _sizes(200, 10, 0), _sizes(200, 10, 3)
    assert rev.ckpt_states == 3 and rev.workspace_bytes < full.workspace_bytes
    assert rev.adjoint_forward_steps > full.adjoint_forward_steps
    with pytest.raises(B.FwiError):
        _sizes(100, 0, 3)
