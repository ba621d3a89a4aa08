"""Pins of the adaptive-step oracle (overlap alpha and its bisection), CPU only."""
import math

import numpy as np
import pytest

from oracle import schedule as S


def test_alpha_at_zero_step_is_one():
    E = np.random.default_rng(0).integers(-100, 100, 500) * 4
    assert S.alpha(E, 0.0) == 1.0


def test_two_level_closed_form():
    n0, n1 = 300, 700
    E = np.array([-8] * n0 + [-4] * n1)
    R = n0 + n1
    for db in (0.01, 0.1, 0.5, 2.0):
        w1 = math.exp(-4 * db)
        W = n0 + n1 * w1
        ref = (n0 * min(1.0, R / W) + n1 * min(1.0, R * w1 / W)) / R
        assert abs(S.alpha(E, db) - ref) < 1e-9


def test_alpha_is_one_minus_total_variation():
    rng = np.random.default_rng(1)
    E = rng.integers(-2000, 0, 3000) * 4
    for db in (0.001, 0.01, 0.05):
        w = np.exp(-db * (E - E.min()).astype(np.float64))
        p = w / w.sum()
        tv = 0.5 * np.abs(p - 1.0 / len(E)).sum()
        assert abs(S.alpha(E, db) - (1 - tv)) < 1e-9


def test_alpha_decreases_with_the_step():
    E = np.random.default_rng(2).normal(-5000, 60, 20000).round().astype(np.int64) * 4
    a = [S.alpha(E, db) for db in np.linspace(0, 0.05, 26)]
    assert all(x >= y - 1e-15 for x, y in zip(a, a[1:]))


def test_exact_overlap_is_the_resampling_overlap():
    """alpha is (1/R) sum_j min(1, tauhat_j) with the resampling's own tauhat (Eq. (3))."""
    from oracle import oracle as O
    E = np.random.default_rng(9).integers(-300, 0, 2000).astype(np.int32) * 4
    for db in (0.002, 0.02):
        _, W, Ssum = O.reweight(E, db)
        tau = O.tau_hat(W, Ssum, len(E))
        assert abs(S.alpha(E, db) - np.minimum(1.0, tau).mean()) < 1e-12


def test_gaussian_energies_closed_form():
    """Normal energies of width sigma: alpha -> 2 Phi(-dbeta sigma / 2) for large R."""
    sigma, R = 40.0, 400000
    E = np.random.default_rng(3).normal(0, sigma, R)
    E = (np.round(E / 4) * 4).astype(np.int64)
    s = E.std()
    for db in (0.005, 0.02, 0.05):
        ref = math.erfc(db * s / 2 / math.sqrt(2))
        assert abs(S.alpha(E, db) - ref) < 0.01


@pytest.mark.parametrize("astar", [0.5, 0.8, 0.95])
def test_step_rule_brackets_the_target(astar):
    E = np.random.default_rng(4).normal(-3000, 50, 5000).round().astype(np.int64) * 4
    dmax = 1.0
    d = S.step_rule(E, astar, dmax, iterations=60)
    A = S.target(astar)
    assert 0.0 <= d < dmax
    assert S.qualifies(E, d, A) and S.alpha(E, d) >= astar - 2.0 ** -32
    assert not S.qualifies(E, d + 1e-12, A)
    # a tiny population spread admits the whole range
    assert S.step_rule(np.full(10, -40), astar, dmax) == dmax


def _population(seed, R=4000):
    return np.random.default_rng(seed).normal(-3000, 40, R).round().astype(np.int64) * 4


@pytest.mark.parametrize("seed", [3, 4])
def test_learned_step_is_exactly_checked_and_near_the_rule(seed):
    """Whatever the proposal, the learned step returns a step with
    alpha >= alpha*; refined from a bracket, it lies within the bracket's
    width / 2^refine below the largest qualifying step (the 200-halving rule:
    alpha falls with the step, so every qualifying step is below it and the
    halving keeps it inside the bracket)."""
    E = _population(seed)
    astar, dmax = 0.7, 0.05
    A = S.target(astar)
    best = S.step_rule(E, astar, dmax, 200)
    for f in (0.3, 0.8, 0.97, 1.0, 1.03, 1.15, 3.0, 40.0):
        cand = f * best
        for bracket, refine in ((1.0, 0), (1.25, 6), (1.25, 12), (2.0, 8)):
            d, fb = S.learned_step(E, cand, astar, dmax, 60, bracket, refine)
            assert S.qualifies(E, d, A), (f, bracket, refine)
            assert d <= best * (1 + 1e-12)
            if fb:
                assert d == S.step_rule(E, astar, dmax, 60)
            elif refine == 0:
                assert d == min(cand, dmax)
            else:
                c = min(cand, dmax)
                lo = c if S.qualifies(E, c, A) else c / bracket
                hi = min(bracket * c, dmax) if S.qualifies(E, c, A) else c
                assert lo <= best <= hi or d == hi
                if lo <= best <= hi and d != hi:  # the bracket holds the best step
                    assert best - d <= (hi - lo) / 2 ** refine * (1 + 1e-12)
        # a proposal within the bracket of the best step never falls back
        if 1 / 1.25 < f <= 1.0 or 1.0 < f < 1.25:
            assert not S.learned_step(E, cand, astar, dmax, 60, 1.25, 6)[1]


def test_learned_step_falls_back_outside_the_bracket_and_for_no_proposal():
    E = _population(5)
    astar, dmax = 0.8, 0.05
    rule = S.step_rule(E, astar, dmax, 60)
    for cand in (0.0, -1.0, 3.0 * rule):
        d, fb = S.learned_step(E, cand, astar, dmax, 60, 1.25, 6)
        assert fb and d == rule
    # dbeta_max itself qualifies: a proposal above it is clamped and kept
    d, fb = S.learned_step(E, 1.0, astar, 1e-6, 60, 1.25, 6)
    assert not fb and d == 1e-6
