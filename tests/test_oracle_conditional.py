"""Pins of the oracle's conditional resampling (the remark of Sec. 3 that the
population may be kept, with importance weights, until their variance grows
too large): weighted reweighting reduces to the plain one for uniform weights;
the effective-sample-size rule on populations whose answer is known; a
population of every state of a small lattice, annealed by kept steps only,
reproduces the exact canonical ln Z and averages; whole conditional anneals
against Kaufman's ln Z (CPU only)."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import exact
from oracle import oracle as O


def test_uniform_log_weights_reduce_to_the_plain_reweighting():
    rng = np.random.default_rng(4)
    for R, dbeta in ((1, 0.3), (1000, 0.0), (1000, 0.004), (5000, 0.07), (300, 2.5)):
        E = (4 * rng.integers(-200, 200, size=R) - 2).astype(np.int32)
        lnQ, W, S = O.reweight(E, dbeta)
        p = O.weighted_reweight(E, np.zeros(R), dbeta)
        assert np.array_equal(p["W"], W) and p["S"] == S
        assert abs(p["lnQ"] - lnQ) <= 1e-12 * max(1.0, abs(lnQ))
        # kept, the population's log-weights are -dbeta (E - E_min) and the largest is 0
        ref = -dbeta * (E.astype(np.float64) - E.min())
        assert np.max(p["lw_next"]) == 0.0
        assert np.allclose(p["lw_next"], ref, rtol=1e-15, atol=0.0)


def test_effective_sample_size_of_known_populations():
    R = 8
    equal = np.full(R, 2 ** 40, np.uint64)
    assert O.ess(equal) == R
    # R equal weights: ESS = R, never below kappa R for kappa <= 1
    assert not O.ess_resamples(equal, O.kappa_units(1.0))[0]
    # k equal non-zero weights among R: ESS = k
    for k in (1, 2, 4, 7):
        W = np.zeros(R, np.uint64)
        W[:k] = 2 ** 40
        assert O.ess(W) == k
        for kappa in (0.0, 0.125, 0.5, 0.875, 1.0):
            assert O.ess_resamples(W, O.kappa_units(kappa))[0] == (k < kappa * R)
    # the comparison is exact at the boundary ESS = kappa R and one unit above it
    W = np.zeros(R, np.uint64)
    W[:4] = 3
    assert not O.ess_resamples(W, O.kappa_units(0.5))[0]
    assert O.ess_resamples(W, O.kappa_units(0.5) + 1)[0]
    # kappa = 0 never resamples; a single dominant weight at kappa R > 1 does
    W = np.array([2 ** 40] + [1] * 99, np.uint64)
    assert not O.ess_resamples(W, 0)[0]
    assert O.ess_resamples(W, O.kappa_units(0.02))[0]
    assert O.kappa_units(0.5) == 32768 and O.kappa_units(1.0) == 65536
    with pytest.raises(ValueError):
        O.kappa_units(1.5)


def enumerated_run(d, L, J):
    """A run whose population is every state of the lattice once (exact at beta = 0)."""
    sigma, E = exact.enumerate_states(d, L, J)
    R = len(E)
    run = O.OracleRun(d, L, R, seed=1, J=J)
    run.import_state(sigma, E.astype(np.int32), np.arange(R, dtype=np.uint32))
    return run, sigma, E


def exact_averages(E, M, beta, N):
    """Canonical <E>/N, <|M|>/N and <M^2>/N^2 over an enumerated state list, in mpmath."""
    keys, cnt = np.unique(np.stack([E, np.abs(M)], axis=1), axis=0, return_counts=True)
    with mp.workdps(40):
        b = mp.mpf(beta)
        w = [mp.mpf(int(c)) * mp.exp(-b * int(k[0])) for k, c in zip(keys, cnt)]
        Z = mp.fsum(w)
        e = mp.fsum(wi * int(k[0]) for wi, k in zip(w, keys)) / Z
        am = mp.fsum(wi * int(k[1]) for wi, k in zip(w, keys)) / Z
        m2 = mp.fsum(wi * int(k[1]) ** 2 for wi, k in zip(w, keys)) / Z
        return float(e) / N, float(am) / N, float(m2) / (N * N)


@pytest.mark.parametrize("glass", [False, True])
def test_kept_steps_over_all_states_give_the_exact_canonical_values(glass):
    """With every state present once and no sweeps, the kept weights are exactly
    the Boltzmann factors, so ln Z_hat (Eq. (7)) and the weighted averages are the
    exact canonical ones at every beta."""
    d, L = 2, 4
    N = L * L
    J = O.ferromagnet(d, L)
    if glass:
        J = np.where(np.random.default_rng(9).random(N * d) < 0.5, -1, 1).astype(np.int8)
    run, sigma, E = enumerated_run(d, L, J)
    M = sigma.astype(np.int64).sum(axis=1)
    dos = exact.brute_force(d, L, J)
    for beta in (0.05, 0.2, 0.35, 0.6, 1.0, 1.5):
        run.reweight(beta)
        R, resampled = run.resample_conditional(O.SYSTEMATIC, 0.0)
        assert not resampled and R == 2 ** N
        ob = run.observables()
        lnZ = exact.lnZ_from_dos(dos, beta)
        assert abs(run.free_energy() - lnZ) < 1e-12 * abs(lnZ)
        e, am, m2 = exact_averages(E, M, beta, N)
        assert ob["weighted"]
        assert abs(ob["e"] - e) < 1e-12
        assert abs(ob["abs_m"] - am) < 1e-12 and abs(ob["m2"] - m2) < 1e-12
        # the plain member averages are those of beta = 0
        assert ob["sumE"] == int(E.sum()) and ob["R"] == 2 ** N
        # ESS = Z(beta)^2 / Z(2 beta) over the states
        ess = math.exp(2 * lnZ - exact.lnZ_from_dos(dos, 2 * beta))
        assert abs(ob["ess"] - ess) < 1e-9 * ess
    assert run.resamplings == 0


def test_kept_steps_telescope():
    """Two kept steps multiply the weights: ln Q_1 + ln Q_2 is the ln Q of one
    reweighting over both, and the log-weights are -(b2 - b0)(E - E_min)."""
    run = O.OracleRun(3, 4, 2000, seed=6)
    run.reweight(0.11)
    run.resample(O.NEAREST_INT)
    run.sweep(3)
    E = run.E.copy()
    b0 = run.beta
    lnq_both, _, _ = O.reweight(E, 0.47 - b0)
    lnq = [run.reweight(0.3)]
    run.resample_conditional(O.NEAREST_INT, 0.0)
    lnq.append(run.reweight(0.47))
    run.resample_conditional(O.NEAREST_INT, 0.0)
    assert abs(sum(lnq) - lnq_both) < 1e-12 * abs(lnq_both)
    ref = -(0.47 - b0) * (E.astype(np.float64) - E.min())
    assert np.allclose(run.log_weights(), ref, rtol=1e-14, atol=1e-14)
    assert run.step == 3 and run.beta == 0.47


def test_resampling_a_weighted_population_draws_by_its_weights():
    """A kept step followed by a resampling: tauhat_j follows the accumulated
    weights exp(lw_j - dbeta E_j), and afterwards the population is uniform."""
    run = O.OracleRun(2, 8, 3000, seed=8)
    run.reweight(0.2)
    run.resample_conditional(O.SYSTEMATIC, 0.0)
    E = run.E.copy()
    lw = run.log_weights()
    run.reweight(0.45)
    W, S = run.pending["W"], run.pending["S"]
    w = np.exp(lw - 0.25 * (E - E.min()))
    tau = O.tau_hat(W, S, run.R)
    assert np.allclose(tau, run.R * w / w.sum(), rtol=1e-9, atol=1e-9)
    R, resampled = run.resample_conditional(O.SYSTEMATIC, 1.0)
    assert resampled and R == run.R and run.lw is None
    assert np.array_equal(np.asarray(run.last_counts), O.counts(O.SYSTEMATIC, W, S, run.R, 8, 0, 2))


def anneal_conditional(run, betas, theta, scheme, kappa):
    kept = 0
    for b in betas[1:]:
        run.reweight(b)
        _, resampled = run.resample_conditional(scheme, kappa)
        kept += 0 if resampled else 1
        run.sweep(theta)
    return kept


def test_conditional_anneal_with_kappa_one_is_the_plain_anneal():
    betas = [0.02 * i for i in range(31)]
    a = O.OracleRun(2, 8, 500, seed=3, run_id=1)
    b = O.OracleRun(2, 8, 500, seed=3, run_id=1)
    kept = anneal_conditional(a, betas, 4, O.POISSON, 1.0)
    for beta in betas[1:]:
        b.reweight(beta)
        b.resample(O.POISSON)
        b.sweep(4)
    assert kept == 0 and a.resamplings == 30
    assert np.array_equal(a.spins, b.spins) and np.array_equal(a.label, b.label)
    assert a.free_energy() == b.free_energy()


@pytest.mark.parametrize("scheme", [O.NEAREST_INT, O.SYSTEMATIC])
def test_conditional_anneal_matches_kaufman(scheme):
    """ln Z_hat of anneals that resample only when ESS < 0.9 R, against the exact
    8x8 ln Z; the population is kept at some steps and resampled at others."""
    L, R, theta = 8, 1000, 10
    betas = [i / 50 for i in range(51)]
    run = O.OracleRun(2, L, R, seed=1, run_id=10 + scheme)
    kept = anneal_conditional(run, betas, theta, scheme, 0.9)
    assert 5 < kept < 45 and run.resamplings == 50 - kept
    err = run.free_energy() - exact.kaufman_lnZ(L, 1.0)
    assert abs(err) < 0.25, err
    ob = run.observables()
    e_exact = exact.kaufman_energy(L, 1.0) / L ** 2
    assert abs(ob["e"] - e_exact) < 0.02
    assert ob["ess"] <= ob["R"]
