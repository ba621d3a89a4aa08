"""Oracle of the adaptive temperature step (test infrastructure only).

The paper names adaptively chosen temperature steps as well established
(Sec. 5) without defining a rule.  Reading used here: the step is chosen so
that the resampling factors of Eq. (1) keep a fixed overlap with the current
population,

    alpha(dbeta) = (1/R) sum_j min(1, tau_j(dbeta)),
    tau_j = R w_j / sum_k w_k,  w_j = exp(-dbeta (E_j - E_min)),

i.e. one minus the total-variation distance between the population and its
reweighted version (alpha(0) = 1, falling with dbeta).  The step is the
largest dbeta in [0, dbeta_max] with alpha >= alpha_star, by bisection with a
fixed number of halvings.  The weights use the decision exponential pa_exp
(the values decide the bisection); sums run over replicas in order.
"""
import numpy as np

from . import oracle as O


def alpha(E, dbeta):
    """Overlap alpha(dbeta) over the population's energies (sums over replicas in order)."""
    E = np.asarray(E, np.int64)
    R = len(E)
    gap = (E - E.min()).astype(np.float64)
    w = O.pa_exp_array(-(float(dbeta) * gap))
    W = float(np.cumsum(w)[-1])                       # sequential sum
    t = np.minimum(1.0, (float(R) * w) / W)
    return float(np.cumsum(t)[-1]) / float(R)


def step_rule(E, alpha_star, dbeta_max, iterations=60):
    """Largest dbeta in [0, dbeta_max] with alpha(dbeta) >= alpha_star (bisection)."""
    if alpha(E, dbeta_max) >= alpha_star:
        return float(dbeta_max)
    lo, hi = 0.0, float(dbeta_max)
    for _ in range(iterations):
        mid = 0.5 * (lo + hi)
        if alpha(E, mid) >= alpha_star:
            lo = mid
        else:
            hi = mid
    return lo
