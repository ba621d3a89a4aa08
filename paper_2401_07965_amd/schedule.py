"""Adaptive-step anneals driven through the C ABI.

``anneal_adaptive`` runs one population-annealing anneal whose temperature
steps come either from the exact overlap rule (pa_step_rule) or from the
learned model with the rule as arbiter and fallback (pa_step_learned); it can
record (features, ln dbeta_rule) pairs for training the model.  Every step
runs in the library's kernels; this module only sequences the calls.
"""
import math
import time

import numpy as np

from . import pa


def anneal_adaptive(run, beta_f, alpha_star, dbeta_max, theta, scheme, mlp=None, record=False,
                    iterations=60, sync=None):
    """Anneal ``run`` (a fresh pa.PARun) from beta 0 to beta_f.

    Returns a dict: steps, lnZ (at beta_f), schedule_s (time spent choosing
    steps), fallbacks, and, if ``record``, X (features) and y (ln dbeta of the
    rule) of every step."""
    beta = 0.0
    steps = fallbacks = 0
    t_sched = 0.0
    X, y = [], []
    run.observables()
    while beta < beta_f:
        if sync:
            sync()
        t0 = time.perf_counter()
        if record:
            X.append(run.features())
        if mlp is None:
            d = run.step_rule(alpha_star, dbeta_max, iterations)
        else:
            d, fb = run.step_learned(mlp, alpha_star, dbeta_max, iterations)
            fallbacks += int(fb)
        t_sched += time.perf_counter() - t0
        if record:
            y.append(math.log(d) if d > 0 else math.log(dbeta_max * 2.0 ** -60))
        if d <= 0.0:
            d = dbeta_max * 2.0 ** -60
        beta = min(beta + d, beta_f)
        run.reweight(beta)
        run.resample(scheme)
        run.sweep(theta)
        run.observables()
        steps += 1
    out = dict(steps=steps, lnZ=run.free_energy(), schedule_s=t_sched, fallbacks=fallbacks)
    if record:
        out["X"] = np.array(X, np.float32)
        out["y"] = np.array(y, np.float32)
    return out


def standardisation(X, y):
    """Input and target means and standard deviations of a training set."""
    xm = X.mean(axis=0)
    xs = X.std(axis=0)
    xs = np.where(xs > 0, xs, 1.0)
    ys = float(y.std()) if float(y.std()) > 0 else 1.0
    return xm.astype(np.float32), xs.astype(np.float32), float(y.mean()), ys
