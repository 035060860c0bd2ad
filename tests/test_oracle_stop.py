"""Pins of the oracle's stopping rule (paper: Methods; a discovery run ends
once its best loss has stood for 500 steps, looked at every 100 steps):
stop steps derived by hand from that rule, and agreement with an
independent window formulation of it."""
import math

import numpy as np
import pytest

import oracle


def test_constant_loss_stops_at_the_first_check_past_patience():
    # step 1 improves on +inf; steps 2..t do not: at t = 500 only 499 steps
    # have passed without improvement, at the next check (600) 599 have
    assert oracle.stop_step([1.0] * 2000) == 600


def test_strictly_decreasing_loss_never_stops():
    assert oracle.stop_step(list(np.linspace(5.0, 1.0, 3000))) is None


def test_last_improvement_sets_the_stop():
    losses = list(np.linspace(5.0, 2.0, 350)) + [2.0] * 1000   # last improvement at step 350
    assert oracle.stop_step(losses) == 900                     # 800: 450 steps, 900: 550 steps
    boundary = list(np.linspace(5.0, 2.0, 100)) + [2.0] * 1000  # last improvement at step 100
    assert oracle.stop_step(boundary) == 600                    # steps 101..600: exactly 500


def test_ties_and_nan_are_no_improvement():
    tie = [1.0] * 2000
    tie[300] = 1.0                                   # equal to the best: not lower
    assert oracle.stop_step(tie) == 600
    nan = [math.nan] * 700 + [0.5] * 10
    assert oracle.stop_step(nan) == 500              # no loss ever improved: 500 steps at step 500


def test_small_patience_and_every_step_checks():
    assert oracle.stop_step([5.0, 4.0, 4.0, 4.0, 4.0, 4.0], patience=3, check_every=1) == 5
    assert oracle.stop_step([5.0, 4.0, 4.0, 3.0, 4.0, 4.0], patience=3, check_every=1) is None


def _window_rule(losses, patience, every):
    # at a check t >= patience, stop iff none of the last `patience` losses is
    # below the best of the losses before them
    for t in range(every, len(losses) + 1, every):
        if t < patience:
            continue
        before = min(losses[:t - patience], default=math.inf)
        if min(losses[t - patience:t]) >= before:
            return t
    return None


@pytest.mark.parametrize("seed", range(6))
def test_matches_window_formulation(seed):
    rng = np.random.default_rng(seed)
    n = 4000
    trend = np.maximum(0.0, 1.0 - np.arange(n) / rng.integers(200, 3000))
    losses = list(trend + rng.random(n) * rng.choice([0.01, 0.3]))
    patience, every = int(rng.choice([50, 200, 500])), int(rng.choice([1, 10, 100]))
    assert oracle.stop_step(losses, patience, every) == _window_rule(losses, patience, every)
