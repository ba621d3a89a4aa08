"""Call sequences that reuse or rebuild what a reweighting prepared or
consumed: the level histogram (built by the sweeps' recount, cleared by the
reweighting after use, rebuilt by the step rule when it is not valid), the
resampling's flags and status (cleared by the reweighting), and the E_min
its weights are counted from.  Every sequence must leave the population, ln Z_hat and the
copy numbers the oracle gives for the same calls."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.paritylib import compare_state, rel_ok

pytestmark = pytest.mark.gpu


def pair(R=500, L=8, seed=4, run_id=0, capacity=None):
    from paper_2401_07965_amd import pa
    cap = capacity if capacity else O.default_capacity(R)
    return (pa.PARun(2, L, R, seed=seed, run_id=run_id, capacity=cap),
            O.OracleRun(2, L, R, seed=seed, run_id=run_id, capacity=cap))


def step_both(g, o, beta, scheme, theta=3):
    assert rel_ok(g.reweight(beta), o.reweight(beta))
    assert g.resample(scheme) == o.resample(scheme)
    g.sweep(theta)
    o.sweep(theta)


@pytest.mark.parametrize("scheme", [O.NEAREST_INT, O.SYSTEMATIC])
def test_observables_and_rule_between_reweight_and_resample(scheme):
    """After a reweighting has cleared the histogram, an observables pass and
    the rule (which rebuilds it, with its own E_min) run before the
    resampling: the resampling still uses the reweighting's weights."""
    print(f"[call orders] observables / rule between reweight and resample, scheme={scheme}", flush=True)
    g, o = pair(run_id=scheme)
    for i, beta in enumerate((0.1, 0.2, 0.3, 0.4, 0.5), 1):
        assert rel_ok(g.reweight(beta), o.reweight(beta))
        g.observables()
        if i % 2 == 0:
            g.step_rule(0.6, 0.2)
            g.features()
        assert g.resample(scheme) == o.resample(scheme)
        g.sweep(3)
        o.sweep(3)
        compare_state(g, o, f"step {i}")
    g.close()


def test_resampling_retried_after_a_capacity_failure():
    """A waiting resampling that overflows leaves the state; a second one with
    another scheme, without a new reweighting, is then applied as the oracle
    applies it."""
    from paper_2401_07965_amd import pa
    print("[call orders] capacity failure, then a retry with another scheme", flush=True)
    g, o = pair(R=64, L=4, seed=5, capacity=64)
    retried = False
    for step in range(40):
        beta = 0.5 * (step + 1)
        assert rel_ok(g.reweight(beta), o.reweight(beta))
        try:
            rg = g.resample(O.POISSON)
        except pa.CapacityError:
            with pytest.raises(O.CapacityError):
                o.resample(O.POISSON)
            assert g.resample(O.SYSTEMATIC) == o.resample(O.SYSTEMATIC) == 64
            retried = True
        else:
            assert rg == o.resample(O.POISSON)
        g.sweep(2)
        o.sweep(2)
        compare_state(g, o, f"step {step}")
        if retried:
            break
    assert retried
    g.close()


def test_repeated_reweighting_and_observables_sequences():
    """Two reweightings in a row (the second replaces the first), observables
    called twice, and steps with no observables at all."""
    print("[call orders] repeated reweighting and observables", flush=True)
    g, o = pair(run_id=7)
    g.reweight(0.9)
    assert rel_ok(g.reweight(0.15), o.reweight(0.15))
    assert g.resample(O.MULTINOMIAL) == o.resample(O.MULTINOMIAL)
    g.sweep(2)
    o.sweep(2)
    g.observables()
    g.observables()
    step_both(g, o, 0.3, O.POISSON)
    step_both(g, o, 0.45, O.SYSTEMATIC)  # no observables since the last step
    g.observables()
    assert rel_ok(g.reweight(0.6), o.reweight(0.6))
    assert rel_ok(g.reweight(0.6), o.reweight(0.6))
    assert g.resample(O.NEAREST_INT) == o.resample(O.NEAREST_INT)
    compare_state(g, o, "end")
    a, b = g.observables(), o.observables()
    assert a["sum_E"] == b["sumE"] and a["families"] == b["families"]
    g.close()


def test_import_then_reweight_uses_the_imported_population():
    """After an import the histogram is rebuilt from the imported energies."""
    from paper_2401_07965_amd import pa
    print("[call orders] import, then reweight", flush=True)
    src, o = pair(run_id=9)
    step_both(src, o, 0.2, O.SYSTEMATIC)
    st = src.export()
    g = pa.PARun(2, 8, 500, seed=4, run_id=9, capacity=O.default_capacity(500))
    g.observables()
    g.import_state(R=st["R"], step=st["step"], sweeps=st["sweeps"], beta=st["beta"], lnZ=st["lnZ"],
                   spins=st["spins"], energy=st["energy"], magnetization=st["magnetization"],
                   label=st["label"])
    assert rel_ok(g.reweight(0.35), o.reweight(0.35))
    assert g.resample(O.NEAREST_INT) == o.resample(O.NEAREST_INT)
    compare_state(g, o, "after import")
    lw, weighted = g.log_weights()
    assert not weighted and np.all(lw == 0.0)
    g.close()
    src.close()


@pytest.mark.parametrize("scheme", [O.SYSTEMATIC, O.POISSON])
def test_histogram_built_by_split_sweeps_cluster_updates_and_no_sweeps(scheme):
    """The sweeps' recount builds the level histogram the next reweighting
    (and the step rule) reads.  Sweeps split over several calls, cluster
    updates between sweeps, steps with no sweep at all, the rule and a
    second reweighting before a resampling: every step ends where the oracle
    does (a histogram counted twice or left stale would change the weights)."""
    print(f"[call orders] split sweeps, cluster updates, empty steps, scheme={scheme}", flush=True)
    g, o = pair(R=700, L=8, seed=9, run_id=scheme)
    plan = [("split", 0.1), ("cluster", 0.2), ("none", 0.25), ("rule", 0.3), ("twice", 0.4), ("split", 0.5),
            ("none", 0.55), ("none", 0.6), ("cluster", 0.7)]
    for i, (kind, beta) in enumerate(plan, 1):
        if kind == "twice":  # a reweighting replaced by a second one
            g.reweight(beta - 0.05)
            o.reweight(beta - 0.05)
        if kind == "rule":
            assert g.step_rule(0.6, 0.2) > 0.0
        assert rel_ok(g.reweight(beta), o.reweight(beta)), i
        assert g.resample(scheme) == o.resample(scheme), i
        if kind == "split":
            for n in (1, 2, 1):
                g.sweep(n)
                o.sweep(n)
        elif kind == "cluster":
            g.sweep(1)
            o.sweep(1)
            g.cluster(1)
            o.cluster(1)
            g.sweep(2)
            o.sweep(2)
        elif kind != "none":
            g.sweep(3)
            o.sweep(3)
        compare_state(g, o, f"step {i} ({kind})")
    g.close()


@pytest.mark.parametrize("scheme", [O.SYSTEMATIC, O.MULTINOMIAL])
def test_resampled_spins_reach_every_reader(scheme):
    """A resampling moves energies, magnetisations and labels at once; its
    spins are taken in by the next sweep's column load, or gathered first
    when something else reads them: an export, a second resampling, cluster
    updates, the overlap, a kept conditional resampling, sweeps split into
    several calls.  Every order gives the oracle's populations."""
    print(f"[call orders] readers of a resampled population, scheme={scheme}", flush=True)
    g, o = pair(R=700, L=8, seed=9, run_id=scheme)
    h, p = pair(R=640, L=8, seed=9, run_id=10 + scheme)
    beta = 0.0

    def resample_both(b):
        assert rel_ok(g.reweight(b), o.reweight(b))
        assert g.resample(scheme) == o.resample(scheme)

    for i in range(1, 9):
        beta += 0.12
        resample_both(beta)
        if i == 1:  # exported before any sweep, then swept
            compare_state(g, o, f"step {i}, after the resampling")
        elif i == 2:  # a second resampling before the sweep
            beta += 0.05
            resample_both(beta)
        elif i == 3:  # cluster updates first
            g.cluster(1)
            o.cluster(1)
        elif i == 4:  # the overlap with another population first
            assert rel_ok(h.reweight(beta), p.reweight(beta))
            assert h.resample(scheme) == p.resample(scheme)
            hist = g.overlap(h)
            R = min(o.Rcur, p.Rcur)
            same = (o.spins[:R] == p.spins[:R]).sum(axis=1)
            assert np.array_equal(hist, np.bincount(same, minlength=o.N + 1))
            h.sweep(1)
            p.sweep(1)
        elif i == 5:  # no sweep: observables, then the next step's reweighting
            g.observables()
            continue
        elif i == 6:  # a conditional resampling that keeps the population
            beta += 0.01
            assert rel_ok(g.reweight(beta), o.reweight(beta))
            assert g.resample_conditional(scheme, 0.0) == o.resample_conditional(scheme, 0.0)
        g.sweep(0)
        g.sweep(1)
        g.sweep(2)
        o.sweep(3)
        compare_state(g, o, f"step {i}")
    compare_state(h, p, "second population")
    g.close()
    h.close()
