"""Pins of the oracle's reweighting and resampling (Sec. 2 step 2, Eq. (1),
Sec. 3, Eq. (3)) by closed forms, exact rationals and sampling statistics."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

SEED, RUN = 3, 0


def random_weights(n, rng, spread=3.0):
    """Integer weights like the ones Q produces: W = floor(2^40 e^{-x}), x >= 0, max 2^40."""
    x = rng.exponential(spread / 3.0, size=n)
    x[rng.integers(n)] = 0.0
    W = np.array([math.floor(math.ldexp(O.pa_exp(-v), 40)) for v in x], dtype=np.uint64)
    return W, int(W.sum(dtype=np.uint64))


def test_reweight_closed_forms():
    rng = np.random.default_rng(0)
    E = rng.integers(-128, 128, size=1000).astype(np.int32)
    lnQ, W, S = O.reweight(E, 0.0)
    assert lnQ == 0.0 and np.all(W == 2 ** 40) and S == 1000 * 2 ** 40
    for dbeta in (0.003, 0.01, 0.2):
        lnQ, W, S = O.reweight(E, dbeta)
        ref = math.log(np.mean(np.exp(-dbeta * E.astype(np.float64))))
        assert abs(lnQ - ref) < 1e-12 * max(1.0, abs(ref))
        emin = int(E.min())
        assert int(W[np.argmin(E)]) == 2 ** 40
        for j in range(0, 1000, 37):
            w = math.exp(-dbeta * (int(E[j]) - emin))
            assert abs(int(W[j]) - w * 2 ** 40) <= 2.0
        assert S == int(W.sum(dtype=np.uint64))
    # no overflow far below the largest double exponent
    E2 = np.array([-40000, -39990, -30000], np.int32)
    lnQ, W, S = O.reweight(E2, 0.05)
    assert math.isfinite(lnQ) and abs(lnQ - (0.05 * 40000 + math.log((1 + math.exp(-0.5)) / 3))) < 1e-9


def exact_tau(W, S, Rt):
    return [Fraction(int(Rt) * int(w), int(S)) for w in W]


@pytest.mark.parametrize("scheme", [O.NEAREST_INT, O.SYSTEMATIC])
def test_low_variance_schemes_take_floor_or_ceil(scheme):
    rng = np.random.default_rng(1)
    for trial in range(20):
        n = int(rng.integers(1, 300))
        W, S = random_weights(n, rng)
        Rt = int(rng.integers(1, 400))
        r = O.counts(scheme, W, S, Rt, SEED, RUN, trial + 1)
        for rj, t in zip(r.tolist(), exact_tau(W, S, Rt)):
            assert math.floor(t) <= rj <= math.ceil(t)


@pytest.mark.parametrize("scheme", [O.MULTINOMIAL, O.SYSTEMATIC])
def test_fixed_size_schemes_keep_R(scheme):
    rng = np.random.default_rng(2)
    for trial in range(30):
        n = int(rng.integers(1, 500))
        W, S = random_weights(n, rng)
        Rt = int(rng.integers(1, 600))
        r = O.counts(scheme, W, S, Rt, SEED, RUN, trial + 1)
        assert int(r.sum()) == Rt
        assert np.all(r[W == 0] == 0)


def test_systematic_matches_direct_point_count():
    """Brute force with exact rationals: points (k + U/2^32) S/R against the boxes."""
    rng = np.random.default_rng(3)
    for trial in range(40):
        n = int(rng.integers(1, 60))
        W, S = random_weights(n, rng)
        Rt = int(rng.integers(1, 80))
        step = trial + 1
        r = O.counts(O.SYSTEMATIC, W, S, Rt, SEED, RUN, step)
        U = int(O.philox(SEED, RUN, [0, 0, step, 7 << 28])[0])
        C = np.concatenate([[0], np.cumsum([int(w) for w in W])]).tolist()
        ref = []
        for j in range(n):
            lo, hi = Fraction(C[j]), Fraction(C[j + 1])
            ref.append(sum(1 for k in range(Rt)
                           if lo <= (k + Fraction(U, 2 ** 32)) * Fraction(S, Rt) < hi))
        assert r.tolist() == ref


def test_multinomial_matches_direct_draws():
    rng = np.random.default_rng(4)
    for trial in range(10):
        n = int(rng.integers(1, 50))
        W, S = random_weights(n, rng)
        Rt = int(rng.integers(1, 100))
        step = trial + 1
        r = O.counts(O.MULTINOMIAL, W, S, Rt, SEED, RUN, step)
        C = np.cumsum([int(w) for w in W]).tolist()
        ref = [0] * n
        for k in range(Rt):
            x = [int(v) for v in O.philox(SEED, RUN, [k, 0, step, 6 << 28])]
            r128 = x[0] + (x[1] << 32) + (x[2] << 64) + (x[3] << 96)
            U = (r128 * S) >> 128
            j = next(i for i in range(n) if C[i] > U)
            ref[j] += 1
        assert r.tolist() == ref


def test_zero_step_is_identity_for_nearest_and_systematic():
    E = np.random.default_rng(5).integers(-50, 50, 777).astype(np.int32)
    _, W, S = O.reweight(E, 0.0)
    for scheme in (O.NEAREST_INT, O.SYSTEMATIC):
        r = O.counts(scheme, W, S, 777, SEED, RUN, 1)
        assert np.all(r == 1)


def sample_counts(scheme, W, S, Rt, trials):
    return np.array([O.counts(scheme, W, S, Rt, SEED, RUN, s + 1) for s in range(trials)],
                    dtype=np.float64)


@pytest.mark.parametrize("scheme", [O.MULTINOMIAL, O.POISSON, O.NEAREST_INT, O.SYSTEMATIC])
def test_unbiased_copy_numbers(scheme):
    """<r_j> = tau_j (Sec. 3), and the variance each scheme implies."""
    rng = np.random.default_rng(6)
    n, Rt, trials = 40, 40, 3000
    W, S = random_weights(n, rng, spread=2.0)
    tau = O.tau_hat(W, S, Rt)
    r = sample_counts(scheme, W, S, Rt, trials)
    mean = r.mean(axis=0)
    f = tau - np.floor(tau)
    if scheme == O.POISSON:
        var = tau
    elif scheme == O.MULTINOMIAL:
        p = tau / Rt
        var = Rt * p * (1 - p)
    else:
        var = f * (1 - f)
    sd = np.sqrt(np.maximum(var, 1e-12) / trials)
    z = (mean - tau) / sd
    # systematic counts are not independent across j but each is unbiased
    assert np.max(np.abs(z[var > 1e-9])) < 5.0
    if scheme != O.SYSTEMATIC:
        emp = r.var(axis=0)
        big = var > 0.05
        assert np.all(np.abs(emp[big] / var[big] - 1) < 0.25)
    else:
        assert np.all(r.var(axis=0) <= f * (1 - f) + 0.05)


def test_variable_size_population_fluctuates_like_sqrt_R():
    rng = np.random.default_rng(7)
    W, S = random_weights(2000, rng)
    for scheme in (O.POISSON, O.NEAREST_INT):
        tot = np.array([O.counts(scheme, W, S, 2000, SEED, RUN, s + 1).sum() for s in range(200)])
        assert abs(tot.mean() - 2000) < 5 * math.sqrt(2000 / 200)
        assert tot.std() < 1.2 * math.sqrt(2000)


def test_multinomial_uniform_weights_family_measure():
    """One multinomial step at equal weights: E[rho_t] = 2 - 1/R."""
    R = 500
    W = np.full(R, 2 ** 40, np.uint64)
    S = R * 2 ** 40
    rho = [float((O.counts(O.MULTINOMIAL, W, S, R, SEED, RUN, s + 1).astype(np.float64) ** 2)
                 .sum()) / R for s in range(400)]
    assert abs(np.mean(rho) - (2 - 1 / R)) < 5 * np.std(rho) / math.sqrt(len(rho))


def test_sampling_variance_order():
    """Eq. (5): nearest-integer and systematic below multinomial below Poisson (Sec. 3)."""
    rng = np.random.default_rng(8)
    W, S = random_weights(1000, rng, spread=1.5)
    tau = O.tau_hat(W, S, 1000)
    sv = {}
    for scheme in (O.MULTINOMIAL, O.POISSON, O.NEAREST_INT, O.SYSTEMATIC):
        r = sample_counts(scheme, W, S, 1000, 50)
        sv[scheme] = float(np.mean((r - tau[None, :]) ** 2))
    assert sv[O.NEAREST_INT] < sv[O.MULTINOMIAL] < sv[O.POISSON]
    assert sv[O.SYSTEMATIC] < sv[O.MULTINOMIAL]


def test_poisson_large_factor_pieces():
    """tauhat above 32 is cut into pieces; the sum stays Poisson(tauhat)."""
    W = np.array([2 ** 40, 1], np.uint64)
    S = 2 ** 40 + 1
    r = sample_counts(O.POISSON, W, S, 100, 2000)[:, 0]
    tau = 100 * (2 ** 40) / S
    assert abs(r.mean() - tau) < 5 * math.sqrt(tau / 2000)
    assert abs(r.var() / tau - 1) < 0.15
