"""Checkpointed reversal schedule of the differentiable rollout (host logic,
no GPU).  Pinned to the closed form of the minimal number of recomputed steps
for binomial checkpointing (Griewank & Walther, ACM TOMS 26 (2000), "revolve"):
with s stored states (the start included) and l steps,
t(l, s) = r l - C(s + r, s + 1), r the smallest integer with C(s + r, s) >= l."""
from math import comb

import pytest

from paper_2405_02483_amd.rollout import reversal_cost, reversal_schedule


def _closed_form(l, s):
    r = 0
    while comb(s + r, s) < l:
        r += 1
    return r * l - comb(s + r, s + 1)


@pytest.mark.parametrize("ncheck", [1, 2, 3, 5])
def test_cost_matches_binomial_closed_form(ncheck):
    s = ncheck + 1
    for l in range(1, 90):
        assert reversal_cost(l, ncheck) == _closed_form(l, s), (l, ncheck)


def test_no_checkpoints_is_quadratic():
    for l in range(1, 30):
        assert reversal_cost(l, 0) == l * (l - 1) // 2


@pytest.mark.parametrize("nsteps,ncheck", [(1, 0), (7, 0), (40, 1), (40, 4), (33, 3), (12, 20)])
def test_schedule_is_a_valid_reversal(nsteps, ncheck):
    acts = reversal_schedule(nsteps, ncheck)
    adj = [a[1] for a in acts if a[0] == "adjoint"]
    assert adj == list(range(nsteps - 1, -1, -1))
    # every advance starts from the start state or from the end of an
    # earlier advance, and never reaches a step already reversed
    reached = {0}
    done = nsteps
    advanced = 0
    for a in acts:
        if a[0] == "advance":
            _, s0, s1 = a
            assert s0 in reached and s0 < s1 < done
            advanced += s1 - s0
            reached.add(s1)
        else:
            assert a[1] in reached or a[1] == 0 or any(
                b[0] == "advance" and b[2] == a[1] for b in acts)
            done = a[1]
    assert advanced == reversal_cost(nsteps, ncheck)
