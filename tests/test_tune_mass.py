"""The heavy-side mass search on model curves sigma(m0) (host logic only)."""
import math

import pytest

from paper_1811_00355_amd.tune_mass import search


def model(mc, slope_heavy=1.0, slope_light=0.8, giveup=None):
    """sigma = slope * |m0 - mc|, the solver giving up (inf) below `giveup`."""
    def f(m):
        if giveup is not None and m < giveup:
            return math.inf
        return slope_heavy * (m - mc) if m >= mc else slope_light * (mc - m)
    return f


@pytest.mark.parametrize("mc,target", [(-0.146, 3e-3), (-0.31, 1e-2), (-0.02, 5e-3), (-0.4, 1e-3)])
def test_search_reaches_the_target_from_the_heavy_side(mc, target):
    seen = search(model(mc), target, 0.0, 0.05, 12)
    m, s = seen[-1]
    assert abs(s / target - 1) <= 0.1 and m > mc          # on the heavy side of the crossing
    assert len(seen) <= 12


def test_search_steps_back_over_a_crossing_and_a_solver_that_gives_up():
    # a secant step that lands past the crossing, where sigma grows again or the solver gives up
    f = model(-0.146, slope_heavy=1.0, slope_light=3.0, giveup=-0.2)
    seen = search(f, 3e-3, 0.0, 0.05, 14)
    m, s = seen[-1]
    assert abs(s / 3e-3 - 1) <= 0.1 and m > -0.146


def test_search_starting_past_the_crossing_moves_up():
    seen = search(model(0.08), 5e-3, 0.0, 0.05, 14)
    assert seen[1][0] < seen[0][0] and any(m > 0.0 for m, _ in seen)
    m, s = seen[-1]
    assert abs(s / 5e-3 - 1) <= 0.1 and m > 0.08


def test_search_respects_the_trial_budget():
    seen = search(lambda m: 1.0 + 0.0 * m, 1e-3, 0.0, 0.05, 5)
    assert len(seen) == 5
