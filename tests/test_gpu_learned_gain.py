"""What the learned step gains over the rule alone, at equal free-energy error.

2D +-J glass, L = 8 (exact ln Z by transfer matrix), R = 2000, beta 0 -> 2:
the model is trained on the GPU from plain rule-driven anneals of six other
disorder samples; on the evaluation sample, 96 independent anneals per
schedule (run_id 0..95), both driven with deferred calls (only the step
choice waits).  The learned step seeds a short exact search with the model's
proposal (bracket 1.25, 6 halvings, the rule as fallback), so both schedules
keep alpha >= alpha* at every step and take steps of nearly the same size.

Asserted, at the statistical resolution of 96 anneals per schedule:
- equal error: the ratio of the mean squared errors of ln Z_hat against the
  exact value lies inside the central 99.8 % of the F(96, 96) law that the
  ratio follows when both schedules have the same (normal) error, and the
  mean errors agree within four standard errors of their difference;
- less time: the learned schedule spends less time choosing steps and less
  wall time in total, with fewer than 5 % of its steps falling back."""
import math
import time

import numpy as np
import pytest

from oracle import exact
from oracle import mlp as Mo
from oracle import oracle as O

pytestmark = pytest.mark.gpu

RUNS = 96


def test_learned_schedule_gain():
    import torch
    from scipy import stats
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
        errs, sched, steps, fb, wall = [], 0.0, 0, 0, 0.0
        for rid in range(RUNS):
            run = pa.PARun(d, L, R, seed=1, run_id=rid, couplings=J)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = anneal_adaptive(run, beta_f, astar, dmax, theta, O.SYSTEMATIC, mlp=model, bracket=1.25,
                                  refine=6, deferred=True, sync=torch.cuda.synchronize)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            errs.append(out["lnZ"] - ref)
            sched += out["schedule_s"]
            steps += out["steps"]
            fb += out["fallbacks"]
            run.close()
        e = np.array(errs)
        res[name] = dict(mse=float(np.mean(e * e)), mean=float(e.mean()), var=float(e.var(ddof=1)),
                         sched=sched, wall=wall, steps=steps, fallbacks=fb)
    print(f"[learned] {res}", flush=True)
    r, l = res["rule"], res["learned"]
    lo, hi = stats.f.ppf(0.001, RUNS, RUNS), stats.f.ppf(0.999, RUNS, RUNS)
    assert lo <= l["mse"] / r["mse"] <= hi, (l["mse"] / r["mse"], lo, hi)
    assert abs(l["mean"] - r["mean"]) <= 4 * math.sqrt((l["var"] + r["var"]) / RUNS)
    assert l["sched"] < r["sched"]
    assert l["wall"] < r["wall"]
    assert l["fallbacks"] < 0.05 * l["steps"]
    mlp.close()
