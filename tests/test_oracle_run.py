"""Pins of whole oracle runs: the free energy of Eq. (7) against exact Z, the
unbiasedness of Q (Eq. (1)), family statistics (Eq. (6)) and the gauge
invariance that ties the +-J glass to the ferromagnet (CPU only)."""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import oracle as O


def schedule(beta_f, points):
    return [i * beta_f / (points - 1) for i in range(points)]


def anneal(run, betas, theta, scheme):
    lnq = []
    for b in betas[1:]:
        lnq.append(run.reweight(b))
        run.resample(scheme)
        run.sweep(theta)
    return lnq


def test_initial_population_observables():
    run = O.OracleRun(2, 8, 1000, seed=1)
    ob = run.observables()
    assert ob["rho_t"] == 1.0 and ob["families"] == 1000
    assert abs(ob["S_f"] - math.log(1000)) < 1e-12
    assert run.free_energy() == 64 * math.log(2.0)


@pytest.mark.parametrize("scheme", [O.NEAREST_INT, O.SYSTEMATIC, O.MULTINOMIAL, O.POISSON])
def test_free_energy_matches_kaufman(scheme):
    """-beta F_hat = ln Z_0 + sum ln Q_k (Eq. (7)) against the exact 8x8 ln Z."""
    L, R, theta = 8, 1000, 10
    betas = schedule(1.0, 51)
    run = O.OracleRun(2, L, R, seed=1, run_id=scheme)
    anneal(run, betas, theta, scheme)
    err = run.free_energy() - exact.kaufman_lnZ(L, 1.0)
    # spread over run_ids at this R is about 0.04 (sd); 6 sd
    assert abs(err) < 0.25, err
    # the final energy per spin is near the exact one at beta = 1
    e_exact = exact.kaufman_energy(L, 1.0) / L ** 2
    assert abs(run.observables()["e"] - e_exact) < 0.02
    ob = run.observables()
    assert 1.0 <= ob["rho_t"] <= ob["R"]


def test_first_Q_is_unbiased():
    """E[Q_1] = Z_{beta_1}/Z_0 for exact beta_0 samples (Eq. (1) with Eq. (7))."""
    L, R = 4, 20000
    dos = exact.brute_force(2, L, O.ferromagnet(2, L))
    for db in (0.1, 0.3):
        run = O.OracleRun(2, L, R, seed=2)
        lnq = run.reweight(db)
        ref = exact.lnZ_from_dos(dos, db) - L * L * math.log(2)
        # relative sd of the mean of exp(-db E): sqrt(Var/R)/mean
        m1 = math.exp(ref)
        m2 = math.exp(exact.lnZ_from_dos(dos, 2 * db) - L * L * math.log(2))
        sd = math.sqrt((m2 - m1 * m1) / R) / m1
        assert abs(lnq - ref) < 5 * sd


def test_product_of_Q_is_unbiased():
    """E[prod_k Q_k] = Z_beta/Z_0 for the fixed-size schemes (a standard SMC property)."""
    L, R = 4, 64
    betas = schedule(0.6, 7)
    ref = exact.lnZ_from_dos(exact.brute_force(2, L, O.ferromagnet(2, L)), 0.6)
    for scheme in (O.SYSTEMATIC, O.MULTINOMIAL):
        ratios = []
        for seed in range(300):
            run = O.OracleRun(2, L, R, seed=100 + seed)
            anneal(run, betas, 2, scheme)
            ratios.append(math.exp(run.free_energy() - ref))
        ratios = np.array(ratios)
        assert abs(ratios.mean() - 1.0) < 5 * ratios.std() / math.sqrt(len(ratios)) + 1e-3


def test_mattis_gauge_reproduces_the_ferromagnet():
    """J(s,mu) = eps_s eps_{s+mu} with spins eps*sigma: identical energies, labels, ln Q."""
    for d, L in ((2, 6), (3, 4)):
        N = L ** d
        rng = np.random.default_rng(d)
        eps = np.where(rng.random(N) < 0.5, -1, 1).astype(np.int8)
        J = np.zeros(N * d, np.int8)
        for mu in range(d):
            nb = exact.neighbor_index(d, L, mu)
            J[np.arange(N) * d + mu] = eps * eps[nb]
        fm = O.OracleRun(d, L, 300, seed=4)
        ea = O.OracleRun(d, L, 300, seed=4, J=J)
        ea.import_state(fm.spins * eps[None, :], fm.E, fm.label)
        for i, b in enumerate(schedule(1.5, 9)[1:]):
            scheme = i % 4
            fm.R = ea.R = 300
            assert fm.reweight(b) == ea.reweight(b)
            assert fm.resample(scheme) == ea.resample(scheme)
            fm.sweep(3)
            ea.sweep(3)
            assert np.array_equal(fm.E, ea.E)
            assert np.array_equal(fm.label, ea.label)
            assert np.array_equal(fm.spins * eps[None, :], ea.spins)
        assert fm.free_energy() == ea.free_energy()


def test_capacity_and_extinction_leave_state_unchanged():
    run = O.OracleRun(2, 4, 100, seed=5, capacity=100)
    run.reweight(0.0)
    # identity resampling keeps 100 replicas, which fits
    assert run.resample(O.NEAREST_INT) == 100
    run.reweight(5.0)
    spins, E = run.spins.copy(), run.E.copy()
    with pytest.raises(O.CapacityError):
        # a huge step concentrates everything; Poisson then overshoots a full capacity
        for s in range(50):
            run.R = 200
            run.resample(O.POISSON)
    assert np.array_equal(run.spins, spins) and np.array_equal(run.E, E)


def test_resample_before_reweight_is_rejected():
    run = O.OracleRun(2, 4, 10, seed=1)
    with pytest.raises(O.PAError):
        run.resample(O.SYSTEMATIC)


def test_extinction_is_an_error_that_leaves_the_state():
    """A single replica under Poisson resampling dies with probability e^-1 per
    step (tauhat = 1); the resampling that would empty the population is
    refused and the replica stays."""
    run = O.OracleRun(2, 4, 1, seed=2, run_id=1)
    died = False
    for s in range(40):
        run.reweight(0.01 * (s + 1))
        spins, E, lnZ = run.spins.copy(), run.E.copy(), run.free_energy()
        try:
            assert run.resample(O.POISSON) >= 1
        except O.ExtinctError:
            died = True
            assert run.Rcur == 1 and np.array_equal(run.spins, spins) and np.array_equal(run.E, E)
            assert run.free_energy() == lnZ
            break
        run.sweep(1)
    assert died  # (1 - e^-1)^40 < 1e-7


def test_family_statistics_closed_forms():
    """rho_t and S_f of label sets whose family sizes are known: one family
    (rho_t = R, S_f = 0), k equal families (rho_t = R / k, S_f = ln k), and
    random sizes against the Shannon entropy of the family fractions as
    scipy computes it and against sum c^2 / R counted directly."""
    from scipy.stats import entropy
    N, R0 = 16, 600
    z = np.zeros(R0, np.int64)
    one = O.population_observables(N, z, z, np.full(R0, 7, np.uint32), R0, 0.0)
    assert one["rho_t"] == R0 and one["S_f"] == 0.0 and one["families"] == 1
    for k in (2, 3, 5, 8):
        lab = np.repeat(np.arange(k, dtype=np.uint32) * 11, R0 // k)
        ob = O.population_observables(N, z[:len(lab)], z[:len(lab)], lab, R0, 0.0)
        assert ob["rho_t"] == len(lab) / k
        assert abs(ob["S_f"] - math.log(k)) < 1e-12
    rng = np.random.default_rng(5)
    for _ in range(5):
        lab = np.sort(rng.integers(0, R0, size=R0).astype(np.uint32))
        ob = O.population_observables(N, z, z, lab, R0, 0.0)
        _, c = np.unique(lab, return_counts=True)
        assert abs(ob["S_f"] - entropy(c / R0)) < 1e-12
        assert ob["rho_t"] == sum(int(x) * int(x) for x in c) / R0
        assert ob["families"] == len(c)
