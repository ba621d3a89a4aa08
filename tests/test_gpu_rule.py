"""GPU parity of the adaptive temperature step (overlap alpha and bisection)."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import schedule as S
from tests.paritylib import compare_state, ea_couplings, rel_ok, run_pair, schedule

pytestmark = pytest.mark.gpu


def test_alpha_and_rule_match_oracle():
    g, o = run_pair(2, 8, 1000, O.NEAREST_INT, schedule(0.4, 5), 5, observables=False)
    for db in (0.0, 0.003, 0.02, 0.1, 0.7):
        a = g.step_alpha(db)
        assert rel_ok(a, S.alpha(o.E, db), 1e-12), (db, a)
    for astar in (0.5, 0.8, 0.95):
        d = g.step_rule(astar, 0.5, 60)
        assert d == S.step_rule(o.E, astar, 0.5, 60), astar
    g.close()


def test_adaptive_anneal_in_lock_step():
    """An anneal whose steps the rule picks: every step chosen identically."""
    from paper_2401_07965_amd import pa
    J = ea_couplings(3, 4, 7)
    g = pa.PARun(3, 4, 500, seed=2, run_id=1, couplings=J)
    o = O.OracleRun(3, 4, 500, seed=2, run_id=1, J=J)
    beta = 0.0
    for step in range(12):
        dg = g.step_rule(0.7, 0.5, 50)
        do = S.step_rule(o.E, 0.7, 0.5, 50)
        assert dg == do, (step, dg, do)
        beta = min(beta + dg, 3.0)
        assert rel_ok(g.reweight(beta), o.reweight(beta))
        assert g.resample(O.SYSTEMATIC) == o.resample(O.SYSTEMATIC)
        g.sweep(4)
        o.sweep(4)
    compare_state(g, o, "adaptive anneal")
    g.close()


def test_rule_full_size_3d():
    """3D +-J L = 16, R = 10^6 (the learned-schedule workload): rule after two steps."""
    from paper_2401_07965_amd import pa
    J = ea_couplings(3, 16, 1)
    g = pa.PARun(3, 16, 1000000, seed=1, run_id=0, couplings=J)
    for b in (0.01, 0.02):
        g.reweight(b)
        g.resample(O.SYSTEMATIC)
        g.sweep(2)
    E = g.export()["energy"]
    for db in (0.001, 0.01):
        assert rel_ok(g.step_alpha(db), S.alpha(E, db), 1e-11)
    assert g.step_rule(0.8, 0.2, 60) == S.step_rule(E, 0.8, 0.2, 60)
    g.close()
