"""GPU parity late in the anneal and at the benchmark workloads' full sizes.

Deep in an anneal the Metropolis thresholds of the high energy-change classes
round to 0 (3D: the class dE = 12 from beta > 1.85, the class dE = 8 from
beta > 2.77; 2D: dE = 8 from beta > 2.77), so the sweep runs its variant
where some classes never accept; and 3D L = 10 cannot use the fixed-axis site
walk.  Here:
- small glasses annealed to beta = 3 against the oracle over the whole
  population at every step (Sec. 2 steps 2-4, Eq. (1));
- full-size populations (2D ferromagnet L = 64, R = 10^5, all four schemes;
  3D +-J L = 10, R = 5 10^5; 3D +-J L = 16, R = 10^6) annealed on the GPU to
  late temperatures, then one step checked: ln Q, copy numbers, labels and
  ln Z_hat over the whole population, spins and energies of sampled replicas;
- the overlap distribution of two full-size L = 10 populations (Figs. 6-7)
  against the oracle's histogram over every pair;
- a batch with the uneven-batch workload's shapes (2D and 3D +-J, L up to
  24) checked on sampled steps against the oracle, the batch's overlap call,
  and replays of the batch's kept HIP graph.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.paritylib import (anneal_deferred, check_step, ea_couplings, rel_ok, run_pair, sample_rows,
                             sampled_step, schedule)

pytestmark = pytest.mark.gpu

SCHEMES = [O.MULTINOMIAL, O.POISSON, O.NEAREST_INT, O.SYSTEMATIC]


@pytest.mark.parametrize("d,L,R,scheme", [(3, 10, 150, O.SYSTEMATIC), (3, 6, 300, O.NEAREST_INT),
                                          (2, 12, 400, O.SYSTEMATIC), (2, 8, 300, O.POISSON)])
def test_glass_anneal_to_beta_3_whole_population(d, L, R, scheme):
    """beta 0 -> 3 in steps of 0.1, theta = 3: every step against the oracle,
    through the beta ranges where classes stop accepting."""
    J = ea_couplings(d, L, 21)
    g, o = run_pair(d, L, R, scheme, schedule(3.0, 31), 3, seed=5, run_id=scheme, J=J)
    assert rel_ok(g.free_energy(), o.free_energy())
    assert O.threshold(3.0, 8) == 0 and O.threshold(2.0, 12) == 0  # the regimes crossed
    g.close()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_2d_L64_R1e5_late_steps(scheme):
    """2D Ising FM, L = 64, R = 10^5, theta = 10, beta_i = 0.6 i/200: the
    steps to beta_147 = 0.441 (near the critical point) and to beta = 0.6."""
    from paper_2401_07965_amd import pa
    betas = schedule(0.6, 201)
    rng = np.random.default_rng(scheme)
    print(f"[parity] 2D L=64 R=1e5 late steps, scheme {scheme}", flush=True)
    g = pa.PARun(2, 64, 100000, seed=1, run_id=scheme)
    anneal_deferred(g, betas[:147], scheme, 10)
    sampled_step(g, 2, 64, None, scheme, betas[147], 10, sample_rows(100000, rng), 1, scheme, 100000)
    anneal_deferred(g, betas[147:200], scheme, 10)
    sampled_step(g, 2, 64, None, scheme, betas[200], 10, sample_rows(100000, rng), 1, scheme, 100000)
    g.close()


def test_3d_L10_R5e5_late_steps():
    """3D +-J L = 10, R = 5 10^5, systematic, beta_i = 3 i/300: the steps to
    beta = 2.0 and 3.0 (classes dE = 12, then dE = 8 never accept)."""
    from paper_2401_07965_amd import pa
    J = ea_couplings(3, 10, 1)
    betas = schedule(3.0, 301)
    rng = np.random.default_rng(7)
    print("[parity] 3D L=10 R=5e5 late steps", flush=True)
    g = pa.PARun(3, 10, 500000, seed=1, run_id=0, couplings=J)
    anneal_deferred(g, betas[:200], O.SYSTEMATIC, 10)
    sampled_step(g, 3, 10, J, O.SYSTEMATIC, betas[200], 10, sample_rows(500000, rng), 1, 0, 500000)
    anneal_deferred(g, betas[200:300], O.SYSTEMATIC, 10)
    sampled_step(g, 3, 10, J, O.SYSTEMATIC, betas[300], 10, sample_rows(500000, rng), 1, 0, 500000)
    g.close()


def test_3d_L16_R1e6_step_at_beta_2():
    """3D +-J L = 16, R = 10^6 (the headline workload), systematic,
    beta_i = 3 i/300: the step to beta = 2.0."""
    from paper_2401_07965_amd import pa
    J = ea_couplings(3, 16, 1)
    betas = schedule(3.0, 301)
    print("[parity] 3D L=16 R=1e6 step to beta 2", flush=True)
    g = pa.PARun(3, 16, 1000000, seed=1, run_id=0, couplings=J)
    anneal_deferred(g, betas[:200], O.SYSTEMATIC, 10)
    sampled_step(g, 3, 16, J, O.SYSTEMATIC, betas[200], 10, sample_rows(1000000, np.random.default_rng(9)),
                 1, 0, 1000000)
    g.close()


def test_3d_L10_two_populations_overlap_full_size():
    """Two populations A, B (run_id 0, 1) of the 3D +-J L = 10 glass, R = 5 10^5
    each, annealed together as a batch to beta = 3 (systematic, theta = 10):
    P(q) from the batch's overlap call equals the oracle's histogram over all
    5 10^5 pairs of the exported states."""
    from paper_2401_07965_amd import pa
    J = ea_couplings(3, 10, 1)
    betas = schedule(3.0, 301)
    cfgs = [dict(dim=3, L=10, R=500000, seed=1, run_id=k, couplings=J) for k in (0, 1)]
    print("[parity] 3D L=10 R=5e5 two populations, overlap", flush=True)
    B = pa.PABatch(cfgs, max_points=len(betas))
    B.anneal(betas, 10, O.SYSTEMATIC, use_graph=True)
    h = B.overlap(0, 1)
    a, b = B.export_run(0), B.export_run(1)
    ref = O.overlap_histogram(a["spins"], b["spins"], a["R"], b["R"], 1000)
    assert h.sum() == 500000
    assert np.array_equal(h, ref)
    # at beta = 3 the populations are far from independent states: |q| well above
    # the N^-1/2 of uncorrelated ones
    q = (2.0 * np.arange(1001) - 1000) / 1000
    assert (h * np.abs(q)).sum() / h.sum() > 0.2
    B.close()


def test_batch_with_uneven_batch_shapes_against_oracle():
    """Runs of the uneven-batch workload's shapes (2D and 3D +-J, L = 8 ... 24,
    theta = 10, beta_i = 3 i/150, systematic) in one batch: the steps to
    beta = 2.0 and beta = 3.0 of every run checked against the oracle (whole
    population for ln Q, copy numbers, labels and ln Z_hat; sampled replicas
    for spins and energies)."""
    from paper_2401_07965_amd import pa
    shapes = [(3, 24, 2000), (2, 24, 3000), (3, 12, 1500), (2, 8, 1000), (2, 16, 800)]
    cfgs = [dict(dim=d, L=L, R=R, seed=1, run_id=k, couplings=ea_couplings(d, L, 1000 + k))
            for k, (d, L, R) in enumerate(shapes)]
    betas = schedule(3.0, 151)
    rng = np.random.default_rng(11)
    B = pa.PABatch(cfgs, max_points=len(betas))
    for k in (99, 149):
        print(f"[parity] uneven batch shapes, step {k} -> {k + 1}", flush=True)
        B.anneal(betas[:k + 1], 10, O.SYSTEMATIC, use_graph=True)
        st0 = [B.export_run(m) for m in range(len(cfgs))]
        B.anneal(betas[:k + 2], 10, O.SYSTEMATIC, use_graph=False)
        rec = B.records()
        for m, c in enumerate(cfgs):
            st1 = B.export_run(m)
            assert st0[m]["step"] == k and st1["step"] == k + 1
            check_step(st0[m], st1, float(rec[m, k + 1]["lnQ"]), int(rec[m, k + 1]["R"]), c["dim"], c["L"],
                       c["couplings"], O.SYSTEMATIC, betas[k + 1], 10, sample_rows(c["R"], rng), 1, m, c["R"])
    B.close()


def test_batch_graph_is_kept_replayed_and_replaced():
    """A batch keeps the graph of its latest anneal: the same anneal again is a
    replay (identical records and states), a different schedule or theta is
    captured anew (equal to the eager anneal), and eager anneals in between
    disturb nothing."""
    from paper_2401_07965_amd import pa
    J = ea_couplings(2, 8, 4)
    cfgs = [dict(dim=2, L=8, R=300, seed=2, run_id=0, couplings=J),
            dict(dim=3, L=4, R=200, seed=2, run_id=1, couplings=ea_couplings(3, 4, 5)),
            dict(dim=2, L=6, R=130, seed=2, run_id=2, couplings=None)]
    A, Bs = schedule(1.5, 10), schedule(2.5, 13)
    B = pa.PABatch(cfgs, max_points=20)

    def run(betas, theta, graph):
        B.anneal(betas, theta, O.SYSTEMATIC, use_graph=graph)
        return B.records().copy(), [B.export_run(m)["spins"] for m in range(len(cfgs))]

    ref_a, sa = run(A, 3, False)
    ref_b, sb = run(Bs, 3, False)
    ref_c, sc = run(A, 2, False)
    for betas, theta, ref, st in ((A, 3, ref_a, sa), (A, 3, ref_a, sa), (Bs, 3, ref_b, sb), (A, 2, ref_c, sc),
                                  (A, 2, ref_c, sc), (A, 3, ref_a, sa)):
        got, gs = run(betas, theta, True)
        assert np.array_equal(got, ref)
        for x, y in zip(gs, st):
            assert np.array_equal(x, y)
        run(Bs[:4], 1, False)  # eager work between
    B.close()


def test_batch_overlap_equals_single_run_overlap():
    from paper_2401_07965_amd import pa
    J = ea_couplings(3, 4, 12)
    betas = schedule(1.0, 6)
    cfgs = [dict(dim=3, L=4, R=300, seed=1, run_id=0, couplings=J),
            dict(dim=3, L=4, R=250, seed=1, run_id=1, couplings=J),
            dict(dim=2, L=8, R=100, seed=1, run_id=2, couplings=None)]
    B = pa.PABatch(cfgs, max_points=len(betas))
    B.anneal(betas, 2, O.NEAREST_INT, use_graph=False)
    h = B.overlap(0, 1)
    ga = pa.PARun(3, 4, 300, seed=1, run_id=0, couplings=J)
    gb = pa.PARun(3, 4, 250, seed=1, run_id=1, couplings=J)
    for g in (ga, gb):
        for b in betas[1:]:
            g.reweight(b)
            g.resample(O.NEAREST_INT)
            g.sweep(2)
    assert np.array_equal(h, ga.overlap(gb))
    a, b = B.export_run(0), B.export_run(1)
    assert np.array_equal(h, O.overlap_histogram(a["spins"], b["spins"], a["R"], b["R"], 64))
    with pytest.raises(pa.PAError):
        B.overlap(0, 2)  # different lattices
    with pytest.raises(pa.PAError):
        B.overlap(0, 3)  # no such run
    ga.close()
    gb.close()
    B.close()
