"""The cluster-update driver on the GPU (Wolff single-cluster updates, the
driver algorithm Sec. 1 names beside local updates): spins, energies,
magnetisations and labels bit-identical to the oracle through anneals that
mix cluster updates and sweeps, 2D and 3D, with and without couplings,
ragged populations; single-spin flips at beta = 0; a sampled full-size step;
lattices beyond the LDS of a workgroup rejected."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.paritylib import compare_observables, compare_state, ea_couplings, rel_ok, rows_from_words, schedule

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,L,R,glass,scheme", [(2, 8, 300, False, O.SYSTEMATIC),
                                                (2, 6, 200, True, O.POISSON),
                                                (2, 16, 130, False, O.NEAREST_INT),
                                                (3, 4, 130, True, O.MULTINOMIAL),
                                                (3, 6, 70, False, O.SYSTEMATIC),
                                                (3, 16, 70, True, O.SYSTEMATIC)])
def test_cluster_anneal_matches_oracle(d, L, R, glass, scheme):
    from paper_2401_07965_amd import pa
    J = ea_couplings(d, L, 3) if glass else None
    print(f"[cluster] d={d} L={L} R={R} glass={glass} scheme={scheme}", flush=True)
    g = pa.PARun(d, L, R, seed=2, run_id=scheme, couplings=J)
    o = O.OracleRun(d, L, R, seed=2, run_id=scheme, J=J)
    for i, beta in enumerate(schedule(1.0 if d == 2 else 0.8, 13)[1:], 1):
        assert rel_ok(g.reweight(beta), o.reweight(beta))
        assert g.resample(scheme) == o.resample(scheme)
        g.cluster(2)
        o.cluster(2)
        g.sweep(1)
        o.sweep(1)
        g.cluster(1)
        o.cluster(1)
        compare_state(g, o, f"step {i}")
    compare_observables(g, o, "end")
    g.close()


def test_cluster_updates_at_beta_zero_flip_one_spin():
    from paper_2401_07965_amd import pa
    g = pa.PARun(2, 8, 150, seed=4)
    o = O.OracleRun(2, 8, 150, seed=4)
    s0 = pa.unpack_spins(g.export()["spins"], 150)
    g.cluster(1)
    o.cluster(1)
    st = compare_state(g, o, "beta = 0")
    assert np.all((pa.unpack_spins(st["spins"], 150) != s0).sum(axis=1) == 1)
    g.close()


def test_cluster_sampled_full_size():
    """2D Ising FM, L = 64, R = 10^5 near beta_c: three cluster updates after a
    few steps, 192 sampled replicas re-updated by the oracle."""
    from paper_2401_07965_amd import pa
    R = 100000
    print("[cluster] 2D L=64 R=1e5 sampled", flush=True)
    g = pa.PARun(2, 64, R, seed=1, run_id=3)
    for beta in (0.1, 0.2, 0.3, 0.4, 0.44):
        g.reweight(beta)
        g.resample(O.SYSTEMATIC)
        g.sweep(2)
    st0 = g.export()
    g.cluster(3)
    st1 = g.export()
    rows = np.concatenate([np.arange(64), np.arange(R - 64, R), np.random.default_rng(3).integers(0, R - 64, 64)])
    rows = np.unique(rows)
    spins = rows_from_words(st0["spins"], rows)
    E = st0["energy"][rows].copy()
    sizes = O.wolff_rows(2, 64, O.ferromagnet(2, 64), rows, spins, E, 1, 3, st0["step"], st0["sweeps"], 3,
                         0.44)
    assert np.array_equal(rows_from_words(st1["spins"], rows), spins)
    assert np.array_equal(st1["energy"][rows], E)
    assert sizes.mean() > 10  # near beta_c the clusters are large
    g.close()


def test_cluster_rejects_lattices_beyond_a_workgroup():
    from paper_2401_07965_amd import pa
    g = pa.PARun(2, 128, 64, seed=1)
    with pytest.raises(pa.PAError):
        g.cluster(1)
    g.sweep(1)  # the run itself is unaffected
    g.close()
