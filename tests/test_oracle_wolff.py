"""Pins of the oracle's cluster-update driver (Wolff single-cluster updates,
the driver algorithm the paper names in Sec. 1), against facts that do not
come from the oracle: at beta = 0 no bond is active, so an update flips one
spin; at bond probability 1 the cluster is a connected component of the
satisfied-bond graph (scipy's connected components); at intermediate beta the
updates leave the Boltzmann distribution of a 4x4 lattice invariant (exact
enumeration, chi-square)."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.stats import chisquare

from oracle import exact
from oracle import oracle as O


def satisfied_components(d, L, J, spins):
    """Component labels of the graph whose edges are the satisfied bonds."""
    N = L ** d
    Jm = np.asarray(J).reshape(N, d)
    idx = np.arange(N)
    rows, cols = [], []
    for mu in range(d):
        nb = exact.neighbor_index(d, L, mu)
        sat = Jm[:, mu] * spins * spins[nb] == 1
        rows.append(idx[sat])
        cols.append(nb[sat])
    r, c = np.concatenate(rows), np.concatenate(cols)
    g = coo_matrix((np.ones(len(r)), (r, c)), shape=(N, N))
    return connected_components(g, directed=False)[1]


@pytest.mark.parametrize("d,L,glass", [(2, 8, False), (3, 4, True)])
def test_beta_zero_flips_one_spin(d, L, glass):
    J = exact_couplings(d, L, glass)
    Jm = J.reshape(L ** d, d)
    o = O.OracleRun(d, L, 300, seed=3, J=J)
    for _ in range(3):
        s0, E0 = o.spins.copy(), o.E.copy()
        sizes = o.cluster(1)
        assert np.all(sizes == 1)
        diff = o.spins != s0
        assert np.all(diff.sum(axis=1) == 1)
        # the energy changes by the single-spin flip's dE = 2 sigma_s h_s
        s = diff.argmax(axis=1)
        for n in range(o.Rcur):
            h = 0
            for mu in range(d):
                up = exact.neighbor_index(d, L, mu)
                dn = np.argsort(up)
                h += Jm[s[n], mu] * s0[n, up[s[n]]] + Jm[dn[s[n]], mu] * s0[n, dn[s[n]]]
            assert o.E[n] - E0[n] == 2 * s0[n, s[n]] * h


@pytest.mark.parametrize("d,L,glass", [(2, 8, False), (2, 6, True), (3, 4, True)])
def test_certain_bonds_flip_a_satisfied_component(d, L, glass):
    J = exact_couplings(d, L, glass)
    assert O.wolff_threshold(400.0) == 1 << 32
    o = O.OracleRun(d, L, 200, seed=5, J=J)
    o.beta = 400.0
    for _ in range(2):
        s0 = o.spins.copy()
        sizes = o.cluster(1)
        for n in range(o.Rcur):
            flipped = np.flatnonzero(o.spins[n] != s0[n])
            comp = satisfied_components(d, L, J, s0[n].astype(np.int64))
            assert len(flipped) == sizes[n, 0]
            assert np.array_equal(flipped, np.flatnonzero(comp == comp[flipped[0]]))


@pytest.mark.parametrize("glass,beta", [(False, 0.4), (True, 0.6)])
def test_updates_keep_the_boltzmann_distribution(glass, beta):
    d, L = 2, 4
    J = exact_couplings(d, L, glass)
    dos = exact.brute_force(d, L, J)
    levels = np.array(sorted(dos))
    w = np.array([dos[e] * np.exp(-beta * (e - levels.min())) for e in levels])
    p = w / w.sum()
    o = O.OracleRun(d, L, 8192, seed=11, J=J)
    o.beta = beta
    o.cluster(40)
    counts = np.array([(o.E == e).sum() for e in levels])
    assert counts.sum() == o.Rcur
    keep = p * o.Rcur >= 5  # chi-square needs populated cells; the rest pooled
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(p[keep], p[~keep].sum()) * o.Rcur
    if exp[-1] == 0:
        obs, exp = obs[:-1], exp[:-1]
    assert chisquare(obs, exp).pvalue > 1e-4
    e_exact = exact.mean_energy_from_dos(dos, beta)
    sd = np.sqrt(((levels - e_exact) ** 2 * p).sum() / o.Rcur)
    assert abs(o.E.mean() - e_exact) < 5 * sd


def exact_couplings(d, L, glass):
    if not glass:
        return O.ferromagnet(d, L)
    rng = np.random.default_rng(17 + d * 10 + L)
    return np.where(rng.random(L ** d * d) < 0.5, -1, 1).astype(np.int8)
