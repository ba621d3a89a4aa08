"""Pins of the oracle's lattice energy, initial sampling and Metropolis sweeps
against brute-force enumeration and exact partition functions (CPU only)."""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import oracle as O


def ea_couplings(d, L, seed):
    rng = np.random.default_rng(seed)
    return np.where(rng.random(L ** d * d) < 0.5, -1, 1).astype(np.int8)


def oracle_dos(d, L, J):
    """Density of states from the oracle's energy function, all 2^N states."""
    N = L ** d
    c = np.arange(2 ** N, dtype=np.int64)[:, None]
    states = (1 - 2 * ((c >> np.arange(N)[None, :]) & 1)).astype(np.int8)
    dos = {}
    for row in states:
        e = O.energy(d, L, J, row)
        dos[e] = dos.get(e, 0) + 1
    return dos


@pytest.mark.parametrize("d,L,kind", [(2, 4, "fm"), (2, 4, "ea"), (3, 2, "fm"), (3, 2, "ea"),
                                      (2, 2, "ea")])
def test_energy_density_of_states_matches_brute_force(d, L, kind):
    J = O.ferromagnet(d, L) if kind == "fm" else ea_couplings(d, L, 11)
    assert oracle_dos(d, L, J) == exact.brute_force(d, L, J)


def test_brute_force_matches_kaufman_and_transfer_matrix():
    """Three independent exact methods agree (4x4 periodic, FM and +-J)."""
    J = O.ferromagnet(2, 4)
    dos = exact.brute_force(2, 4, J)
    for beta in (0.1, 0.3, 0.44068, 0.7, 1.3):
        lz = exact.lnZ_from_dos(dos, beta)
        assert abs(lz - exact.kaufman_lnZ(4, beta)) < 1e-12
        assert abs(lz - exact.transfer_matrix_lnZ(4, J, beta)) < 1e-12
    Jr = ea_couplings(2, 4, 5)
    dos = exact.brute_force(2, 4, Jr)
    for beta in (0.2, 0.9, 2.5):
        assert abs(exact.lnZ_from_dos(dos, beta) - exact.transfer_matrix_lnZ(4, Jr, beta)) < 1e-11
    # larger: Kaufman against the transfer matrix at L = 6, 8
    for L in (6, 8):
        for beta in (0.3, 0.5):
            assert abs(exact.kaufman_lnZ(L, beta) -
                       exact.transfer_matrix_lnZ(L, O.ferromagnet(2, L), beta)) < 1e-10


def test_kaufman_energy_and_specific_heat_match_brute_force():
    """e and c from central differences of Kaufman's ln Z equal the moments of the
    enumerated 4x4 density of states."""
    dos = exact.brute_force(2, 4, O.ferromagnet(2, 4))
    for beta in (0.1, 0.3, 0.44068, 0.7):
        e, c = exact.kaufman_e_c(4, beta)
        m1, var = exact.moments_from_dos(dos, beta)
        assert abs(e - m1 / 16) < 1e-12
        assert abs(c - beta * beta * var / 16) < 1e-10


def test_paper_critical_point(golden):
    """The exact specific heat peak approaches the beta_c the paper prints (Sec. 3)."""
    bc = golden["beta_c_2d_ising"]["value"]
    assert abs(exact.beta_c() - bc) < 1e-5  # printed to five decimals
    # finite-L specific heat from Kaufman's ln Z peaks close to beta_c
    L = 32
    import mpmath as mp
    betas = np.linspace(0.40, 0.46, 61)
    h = mp.mpf("1e-8")
    c = []
    for b in betas:
        b = mp.mpf(b)
        f0 = exact.kaufman_lnZ_mp(L, b)
        fp = exact.kaufman_lnZ_mp(L, b + h)
        fm = exact.kaufman_lnZ_mp(L, b - h)
        c.append(float(b * b * (fp - 2 * f0 + fm) / (h * h)) / L ** 2)
    peak = betas[int(np.argmax(c))]
    assert abs(peak - bc) < 0.01


def test_ground_and_antiferro_states():
    for d, L in ((2, 4), (2, 6), (3, 4), (3, 2)):
        N = L ** d
        J = O.ferromagnet(d, L)
        assert O.energy(d, L, J, np.ones(N, np.int8)) == -d * N
        g = exact.site_grid(d, L)
        parity = sum(np.indices(g.shape)).reshape(-1) % 2
        assert O.energy(d, L, J, (1 - 2 * parity).astype(np.int8)) == d * N


def test_init_is_iid_uniform():
    d, L, R = 2, 8, 4096
    spins, E, label = O.init_rows(d, L, np.arange(R), 1, 0, O.ferromagnet(d, L))
    assert np.array_equal(label, np.arange(R))
    assert set(np.unique(spins).tolist()) == {-1, 1}
    N = L ** d
    # E is a sum of dN independent +-1 bond terms at beta = 0: mean 0, variance dN
    assert abs(E.mean()) < 5 * math.sqrt(d * N / R)
    assert abs(E.var() / (d * N) - 1.0) < 0.1
    assert abs((spins == -1).mean() - 0.5) < 5 * 0.5 / math.sqrt(R * N)
    for n in (0, 17, 4095):
        assert E[n] == O.energy(d, L, O.ferromagnet(d, L), spins[n])
    # a sample of rows equals the same rows of the full population
    rows = np.array([3, 64, 65, 1000])
    s2, e2, l2 = O.init_rows(d, L, rows, 1, 0, O.ferromagnet(d, L))
    assert np.array_equal(s2, spins[rows]) and np.array_equal(e2, E[rows])
    # another run_id draws another population
    s3, _, _ = O.init_rows(d, L, np.arange(64), 1, 1, O.ferromagnet(d, L))
    assert not np.array_equal(s3, spins[:64])


@pytest.mark.parametrize("d,L", [(2, 4), (2, 6), (3, 4)])
def test_beta_zero_sweep_flips_every_spin(d, L):
    J = ea_couplings(d, L, 2)
    spins, E, _ = O.init_rows(d, L, np.arange(130), 3, 0, J)
    s0 = spins.copy()
    O.sweep_rows(d, L, J, np.arange(130), spins, E, 3, 0, 1, 0, 1, 0.0)
    assert np.array_equal(spins, -s0)


@pytest.mark.parametrize("d,L,kind", [(2, 6, "fm"), (2, 8, "ea"), (3, 4, "ea"), (3, 2, "fm")])
def test_tracked_energy_equals_recomputed(d, L, kind):
    J = O.ferromagnet(d, L) if kind == "fm" else ea_couplings(d, L, 9)
    R = 200
    spins, E, _ = O.init_rows(d, L, np.arange(R), 5, 0, J)
    for step, beta in enumerate((0.2, 0.5, 1.0, 2.0), start=1):
        O.sweep_rows(d, L, J, np.arange(R), spins, E, 5, 0, step, 0, 3, beta)
        for n in range(0, R, 7):
            assert E[n] == O.energy(d, L, J, spins[n])


def test_zero_temperature_never_raises_energy():
    d, L, R = 2, 8, 128
    J = ea_couplings(d, L, 4)
    spins, E, _ = O.init_rows(d, L, np.arange(R), 1, 0, J)
    for t in range(10):
        before = E.copy()
        O.sweep_rows(d, L, J, np.arange(R), spins, E, 1, 0, 1, t, 1, 60.0)
        assert np.all(E <= before)


@pytest.mark.parametrize("d,L,kind,beta", [(2, 4, "fm", 0.4), (2, 4, "ea", 0.8),
                                           (3, 2, "fm", 0.3)])
def test_sweeps_sample_boltzmann(d, L, kind, beta):
    """Many replicas after many sweeps follow g(E) exp(-beta E)/Z (brute force)."""
    J = O.ferromagnet(d, L) if kind == "fm" else ea_couplings(d, L, 21)
    R = 8192
    rows = np.arange(R)
    spins, E, _ = O.init_rows(d, L, rows, 7, 0, J)
    O.sweep_rows(d, L, J, rows, spins, E, 7, 0, 1, 0, 60, beta)
    dos = exact.brute_force(d, L, J)
    levels = sorted(dos)
    lz = exact.lnZ_from_dos(dos, beta)
    p = np.array([dos[e] * math.exp(-beta * e - lz) for e in levels])
    obs = np.array([(E == e).sum() for e in levels], dtype=np.float64)
    exp_cnt = p * R
    keep = exp_cnt > 5
    chi2 = float((((obs - exp_cnt) ** 2)[keep] / exp_cnt[keep]).sum())
    dof = int(keep.sum()) - 1
    # chi^2 with dof degrees of freedom: mean dof, sd sqrt(2 dof)
    assert chi2 < dof + 6 * math.sqrt(2 * dof) + 10, (chi2, dof)


@pytest.mark.parametrize("d,L,kind,beta", [(2, 4, "fm", 0.4), (2, 4, "ea", 0.8)])
def test_population_energy_moments_match_exact(d, L, kind, beta):
    """The observables' <E>, <E^2>, <E^3> of an equilibrated population agree with
    the exact canonical moments from the density of states (brute force) within
    six standard errors; a dropped term or a wrong power fails this."""
    J = O.ferromagnet(d, L) if kind == "fm" else ea_couplings(d, L, 21)
    R = 8192
    N = L ** d
    rows = np.arange(R)
    spins, E, _ = O.init_rows(d, L, rows, 9, 0, J)
    O.sweep_rows(d, L, J, rows, spins, E, 9, 0, 1, 0, 60, beta)
    M = spins.astype(np.int64).sum(axis=1)
    obs = O.population_observables(N, E, M, np.arange(R, dtype=np.uint32), R, 0.0)
    dos = exact.brute_force(d, L, J)
    lz = exact.lnZ_from_dos(dos, beta)
    mom = {k: sum(g * e ** k * math.exp(-beta * e - lz) for e, g in dos.items()) for k in range(7)}
    for k, key, scale in ((1, "e", N), (2, "e2", N ** 2), (3, "e3", N ** 3)):
        sd = math.sqrt((mom[2 * k] - mom[k] ** 2) / R)
        assert abs(obs[key] * scale - mom[k]) < 6 * sd + 1e-9, (k, obs[key] * scale, mom[k], sd)
    # the exact integer sums behind them
    assert obs["sumE3"] == sum(int(e) ** 3 for e in E.tolist())


def test_plane_pair_count_of_all_drawing_words():
    """Work count of the sweeps: a word-site whose 64 replicas all draw needs
    plane pairs up to its slowest replica's deciding plane; each plane decides
    a replica with probability 1/2, so E[pairs] = sum_{p=1..16} P(max_b k_b >=
    2(p-1)) = sum_p 1 - (1 - 2^(-2(p-1)))^64.  A ferromagnet's ordered state
    at beta = 0.5 keeps (nearly) every replica drawing."""
    d, L, R = 2, 16, 64
    J = O.ferromagnet(d, L)
    spins = np.ones((R, L * L), np.int8)
    E = np.full(R, -2 * L * L, np.int32)
    theta = 40
    calls = O.sweep_rows(d, L, J, np.arange(R), spins, E, 21, 0, 1, 0, theta, 0.5)
    expect = sum(1.0 - (1.0 - 2.0 ** (-2 * (p - 1))) ** 64 for p in range(1, 17))
    per_site = calls / (theta * L * L)
    assert abs(per_site - expect) < 0.05, (per_site, expect)
    # nothing draws at beta = 0 (every move accepted) or when no move can be accepted
    spins = np.ones((R, L * L), np.int8)
    assert O.sweep_rows(d, L, J, np.arange(R), spins, E.copy(), 21, 0, 1, 0, 2, 0.0) == 0
    spins = np.ones((R, L * L), np.int8)
    assert O.sweep_rows(d, L, J, np.arange(R), spins, E.copy(), 21, 0, 1, 0, 2, 1e4) == 0
