"""What the learned step gains over the rule alone, at equal free-energy error.

2D +-J glass, L = 8 (exact ln Z by transfer matrix), R = 2000: the model is
trained on the GPU from plain rule-driven anneals of six other disorder
samples; on the evaluation sample, 8 independent anneals per schedule.  Both
schedules keep the overlap alpha >= alpha* at every step (the learned one
through the exact overlap check), so their free-energy errors must agree within the
run-to-run spread, while the learned one spends less time choosing steps."""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import mlp as Mo
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def test_learned_schedule_gain():
    from paper_2401_07965_amd import pa, workloads
    from paper_2401_07965_amd.schedule import anneal_adaptive, standardisation
    d, L, R, theta, beta_f, astar, dmax = 2, 8, 2000, 5, 2.0, 0.7, 0.25
    Xs, ys = [], []
    for s in range(2, 8):
        run = pa.PARun(d, L, R, seed=1, run_id=0, couplings=workloads.pm_j_couplings(d, L, s))
        out = anneal_adaptive(run, beta_f, astar, dmax, theta, O.SYSTEMATIC, record=True)
        Xs.append(out["X"])
        ys.append(out["y"])
        run.close()
    X, y = np.concatenate(Xs), np.concatenate(ys)
    xm, xs, ym, ysd = standardisation(X, y)
    mlp = pa.PAMlp(Mo.init_params(0), xm, xs, ym, ysd, max_samples=len(y))
    mlp.set_data(X, y)
    loss = mlp.train(1500, 3e-3)
    print(f"[learned] {len(y)} training steps, final loss {loss:.4f}", flush=True)
    J = workloads.pm_j_couplings(d, L, 1)
    ref = exact.transfer_matrix_lnZ(L, J, beta_f)
    res = {}
    for name, model in (("rule", None), ("learned", mlp)):
        errs, sched, steps, fb = [], 0.0, 0, 0
        for rid in range(8):
            run = pa.PARun(d, L, R, seed=1, run_id=rid, couplings=J)
            out = anneal_adaptive(run, beta_f, astar, dmax, theta, O.SYSTEMATIC, mlp=model)
            errs.append(out["lnZ"] - ref)
            sched += out["schedule_s"]
            steps += out["steps"]
            fb += out["fallbacks"]
            run.close()
        res[name] = dict(rmsd=math.sqrt(np.mean(np.square(errs))), sched=sched, steps=steps,
                         fallbacks=fb)
    print(f"[learned] {res}", flush=True)
    assert res["learned"]["rmsd"] <= 1.5 * res["rule"]["rmsd"] + 0.05
    assert res["learned"]["sched"] < res["rule"]["sched"]
    assert res["learned"]["fallbacks"] < 0.5 * res["learned"]["steps"]
    mlp.close()
