"""Conditional resampling on the GPU (the remark of Sec. 3 that the population
may be kept, with importance weights, while their variance is small): every
decision, member, log-weight and copy number bit-identical to the oracle, ln Q,
ln Z_hat and the weighted averages to 1e-10; deferred calls; kappa = 1 is the
plain resampling; a population of every state of a 4x4 lattice reproduces the
exact ln Z and averages through kept steps."""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import oracle as O
from tests.paritylib import compare_state, ea_couplings, rel_ok, schedule

pytestmark = pytest.mark.gpu


def compare_weighted(g, o, where):
    """Members (bit-exact), log-weights (bit-exact) and the averages."""
    compare_state(g, o, where)
    lw, weighted = g.log_weights()
    assert weighted == (o.lw is not None), where
    assert np.array_equal(lw, o.log_weights()), f"log-weights differ {where}"
    a, b = g.observables(), o.observables()
    assert a["weighted"] == b["weighted"] and a["R"] == b["R"], where
    assert a["sum_E"] == b["sumE"] and a["sum_E3"] == b["sumE3"] and a["sum_c2"] == b["sumC2"], where
    for k in ("e", "e2", "e3", "abs_m", "m2", "ess", "rho_t", "S_f"):
        assert rel_ok(a[k], b[k]) or abs(a[k] - b[k]) < 1e-12, (k, a[k], b[k], where)
    assert a["sv"] == b["sv"] or rel_ok(a["sv"], b["sv"], 1e-9), (a["sv"], b["sv"], where)


def conditional_pair(d, L, R, scheme, betas, theta, kappa, seed=1, run_id=0, J=None):
    from paper_2401_07965_amd import pa
    cap = O.default_capacity(R)
    print(f"[conditional] d={d} L={L} R={R} scheme={scheme} kappa={kappa} steps={len(betas) - 1}",
          flush=True)
    g = pa.PARun(d, L, R, seed=seed, run_id=run_id, capacity=cap, couplings=J)
    o = O.OracleRun(d, L, R, seed=seed, run_id=run_id, J=J, capacity=cap)
    decisions = []
    for i, b in enumerate(betas[1:], 1):
        qg, qo = g.reweight(b), o.reweight(b)
        assert rel_ok(qg, qo), (i, qg, qo)
        rg, ro = g.resample_conditional(scheme, kappa), o.resample_conditional(scheme, kappa)
        assert rg == ro, (i, rg, ro)
        decisions.append(rg[1])
        g.sweep(theta)
        o.sweep(theta)
        compare_weighted(g, o, f"step {i}")
    assert g.counters()["resamplings"] == o.resamplings == sum(decisions)
    return g, o, decisions


@pytest.mark.parametrize("scheme", [O.MULTINOMIAL, O.POISSON, O.NEAREST_INT, O.SYSTEMATIC])
def test_conditional_anneal_matches_oracle(scheme):
    g, o, dec = conditional_pair(2, 8, 700, scheme, schedule(1.0, 41), 5, 0.9, seed=3,
                                 run_id=scheme)
    assert 0 < sum(dec) < len(dec)  # both branches taken, resamplings of weighted populations
    assert any(not a and b for a, b in zip(dec, dec[1:]))
    g.close()


def test_conditional_glass_several_chunks():
    """3D +-J glass, R spanning three 1024-replica chunks with a ragged tail."""
    J = ea_couplings(3, 6, 21)
    g, o, dec = conditional_pair(3, 6, 2500, O.SYSTEMATIC, schedule(1.5, 31), 3, 0.8, seed=7,
                                 run_id=2, J=J)
    assert 0 < sum(dec) < len(dec)
    g.close()


def test_deferred_conditional_matches_waiting_calls():
    from paper_2401_07965_amd import pa
    d, L, R = 2, 8, 700
    betas = schedule(1.0, 41)
    print("[conditional] deferred d=2 L=8 R=700 nearest kappa=0.9", flush=True)
    a = pa.PARun(d, L, R, seed=5, run_id=1)
    b = pa.PARun(d, L, R, seed=5, run_id=1)
    o = O.OracleRun(d, L, R, seed=5, run_id=1)
    for beta in betas[1:]:
        assert a.reweight(beta, wait=False) is None
        assert a.resample_conditional(O.NEAREST_INT, 0.9, wait=False) is None
        a.sweep(4)
        assert a.observables(wait=False) is None
        b.reweight(beta)
        b.resample_conditional(O.NEAREST_INT, 0.9)
        b.sweep(4)
        b.observables()
        o.reweight(beta)
        o.resample_conditional(O.NEAREST_INT, 0.9)
        o.sweep(4)
    sa, sb = a.export(), b.export()
    for k in ("spins", "energy", "magnetization", "label"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["lnZ"] == sb["lnZ"] and sa["R"] == sb["R"]
    assert np.array_equal(a.log_weights()[0], b.log_weights()[0])
    assert a.observables() == b.observables()
    assert a.counters() == b.counters()
    compare_weighted(a, o, "deferred end")
    a.close()
    b.close()


def test_kappa_one_is_the_plain_resampling():
    from paper_2401_07965_amd import pa
    print("[conditional] kappa=1 against pa_resample, 2D L=16 R=3000 Poisson", flush=True)
    a = pa.PARun(2, 16, 3000, seed=2, run_id=4)
    b = pa.PARun(2, 16, 3000, seed=2, run_id=4)
    for beta in schedule(0.6, 21)[1:]:
        a.reweight(beta)
        ra, done = a.resample_conditional(O.POISSON, 1.0)
        assert done
        b.reweight(beta)
        assert b.resample(O.POISSON) == ra
        a.sweep(3)
        b.sweep(3)
    sa, sb = a.export(), b.export()
    for k in ("spins", "energy", "magnetization", "label"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["lnZ"] == sb["lnZ"]
    oa, ob = a.observables(), b.observables()
    assert not oa["weighted"] and oa == ob
    a.close()
    b.close()


def test_kept_steps_over_all_states_give_exact_values():
    """Every state of the 4x4 ferromagnet once (R = 65536, exact at beta = 0),
    kappa = 0 and no sweeps: ln Z_hat and the weighted averages are the exact
    canonical ones, ESS = Z(beta)^2 / Z(2 beta)."""
    from paper_2401_07965_amd import pa
    d, L = 2, 4
    N = L * L
    J = O.ferromagnet(d, L)
    sigma, E = exact.enumerate_states(d, L, J)
    R = len(E)
    M = sigma.astype(np.int64).sum(axis=1)
    print(f"[conditional] all {R} states of the 4x4 ferromagnet, kept steps", flush=True)
    g = pa.PARun(d, L, R, seed=1, capacity=R)
    g.import_state(R=R, step=0, sweeps=0, beta=0.0, lnZ=N * math.log(2.0), spins=pa.pack_spins(sigma),
                   energy=E.astype(np.int32), magnetization=M.astype(np.int32),
                   label=np.arange(R, dtype=np.uint32))
    dos = exact.brute_force(d, L, J)
    for beta in (0.1, 0.3, 0.44, 0.7, 1.2):
        g.reweight(beta)
        assert g.resample_conditional(O.SYSTEMATIC, 0.0) == (R, False)
        lnZ = exact.lnZ_from_dos(dos, beta)
        assert abs(g.free_energy() - lnZ) < 1e-10 * abs(lnZ)
        ob = g.observables()
        assert ob["weighted"]
        assert abs(ob["e"] - exact.mean_energy_from_dos(dos, beta) / N) < 1e-10
        ess = math.exp(2 * lnZ - exact.lnZ_from_dos(dos, 2 * beta))
        assert abs(ob["ess"] - ess) < 1e-9 * ess
        w = np.exp(-beta * (E - E.min()).astype(np.float64))
        assert abs(ob["m2"] - float(np.sum(w * M * M) / w.sum()) / N ** 2) < 1e-10
    with pytest.raises(pa.StateError):
        g.step_rule(0.5, 0.1)  # the overlap rule needs a uniform population
    g.reweight(1.3)
    rn, done = g.resample_conditional(O.SYSTEMATIC, 1.0)
    assert done and rn == R and not g.log_weights()[1]
    assert g.step_rule(0.5, 0.1) > 0.0
    g.close()


def test_deferred_conditional_failure_freezes_with_weights_intact():
    """A kept step, then a resampling that overflows the capacity (deferred):
    the run freezes with the kept members and their log-weights unchanged."""
    from paper_2401_07965_amd import pa
    print("[conditional] capacity failure after a kept step, L=4 R=64 capacity=64", flush=True)
    o = O.OracleRun(2, 4, 64, seed=5, capacity=64)
    o.reweight(0.05)
    assert o.resample_conditional(O.POISSON, 0.0) == (64, False)
    fail = None
    for step in range(30):
        o.reweight(0.05 + 0.5 * (step + 1))
        try:
            o.resample_conditional(O.POISSON, 1.0)
        except O.CapacityError:
            fail = step
            break
        o.sweep(2)
    assert fail is not None
    g = pa.PARun(2, 4, 64, seed=5, capacity=64)
    g.reweight(0.05)
    g.resample_conditional(O.POISSON, 0.0)
    for step in range(fail + 2):
        g.reweight(0.05 + 0.5 * (step + 1), wait=False)
        g.resample_conditional(O.POISSON, 1.0, wait=False)
        g.sweep(2)
    with pytest.raises(pa.CapacityError):
        g.free_energy()
    st = g.export()
    assert st["R"] == o.Rcur and np.array_equal(st["energy"], o.E)
    assert np.array_equal(pa.unpack_spins(st["spins"], st["R"]), o.spins)
    lw, weighted = g.log_weights()
    assert weighted == (o.lw is not None) and np.array_equal(lw, o.log_weights())
    g.close()
