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


class NoStepError(RuntimeError):
    """The step rule found no positive temperature step."""


def anneal_adaptive(run, beta_f, alpha_star, dbeta_max, theta, scheme, mlp=None, record=False,
                    iterations=60, sync=None, max_steps=100000, bracket=1.0, refine=0, deferred=False):
    """Anneal ``run`` (a fresh pa.PARun) from beta 0 to beta_f.

    Each step's dbeta comes from the overlap rule or, with ``mlp``, from the
    learned step (its proposal checked exactly, refined in ``bracket`` with
    ``refine`` halvings, the rule as fallback).  With ``deferred`` the
    reweighting, resampling and observables of a step are enqueued without
    waiting; only the step choice waits for the device.  ``sync`` (if given)
    runs before each step choice is timed.

    Returns a dict: steps, lnZ (at beta_f), schedule_s (time spent choosing
    steps), fallbacks, betas (the schedule taken) and, if ``record``, X
    (features) and y (ln dbeta of the rule) of every step.

    Raises NoStepError when the rule returns no step that moves beta (too few
    bisection iterations to resolve a qualifying step: only dbeta = 0 is
    certain to qualify) or when more than ``max_steps`` steps would be needed."""
    beta = 0.0
    steps = fallbacks = 0
    t_sched = 0.0
    X, y = [], []
    betas = [0.0]
    run.observables()
    while beta < beta_f:
        if steps >= max_steps:
            raise NoStepError(f"beta {beta} after {steps} steps: more than max_steps = {max_steps}")
        if sync:
            sync()
        t0 = time.perf_counter()
        if record:
            X.append(run.features())
        if mlp is None:
            d = run.step_rule(alpha_star, dbeta_max, iterations)
        else:
            d, fb = run.step_learned(mlp, alpha_star, dbeta_max, iterations, bracket, refine)
            fallbacks += int(fb)
        t_sched += time.perf_counter() - t0
        nxt = min(beta + d, beta_f) if d > 0.0 else beta
        if nxt <= beta:
            raise NoStepError(f"the step rule returned dbeta = {d} at beta = {beta} "
                              f"({iterations} bisection iterations); no step moves beta")
        if record:
            y.append(math.log(d))
        beta = nxt
        betas.append(beta)
        run.reweight(beta, wait=not deferred)
        run.resample(scheme, wait=not deferred)
        run.sweep(theta)
        run.observables(wait=not deferred)
        steps += 1
    out = dict(steps=steps, lnZ=run.free_energy(), schedule_s=t_sched, fallbacks=fallbacks, betas=betas)
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
