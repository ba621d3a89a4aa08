"""Oracle of the adaptive temperature step (test infrastructure only).

The paper names adaptively chosen temperature steps as well established
(Sec. 5) without defining a rule.  Reading used here: the step is chosen so
that the resampling factors of Eq. (1) keep a fixed overlap with the current
population,

    alpha(dbeta) = (1/R) sum_j min(1, tau_j(dbeta)),   tau_j = R W_j / S,

i.e. one minus the total-variation distance between the population and its
reweighted version (alpha(0) = 1, falling with dbeta).  The factors are the
ones the resampling itself uses: the integer weights W_j = floor(2^40
pa_exp(-dbeta (E_j - E_min))) and S = sum_j W_j, so alpha is the exact
rational sum_j min(S, R W_j) / (R S).  The step is the largest dbeta in
[0, dbeta_max] with alpha >= alpha_star, by bisection with a fixed number of
halvings; alpha_star is taken to 2^-32 (A = nearest integer to 2^32
alpha_star, ties to even) and the test alpha >= alpha_star is the exact
integer comparison 2^32 sum_j min(S, R W_j) >= A R S.
"""
import math
from fractions import Fraction

import numpy as np

from . import oracle as O


def overlap_fraction(E, dbeta):
    """(numerator, denominator) of alpha(dbeta), exact integers."""
    E = np.asarray(E, np.int32)
    R = len(E)
    _, W, S = O.reweight(E, dbeta)
    m = np.minimum(np.uint64(S), W * np.uint64(R))  # R W_j < 2^64
    num = int((m >> np.uint64(32)).sum(dtype=np.uint64)) * 2 ** 32 + \
        int((m & np.uint64(0xFFFFFFFF)).sum(dtype=np.uint64))
    return num, R * int(S)


def alpha(E, dbeta):
    num, den = overlap_fraction(E, dbeta)
    return float(Fraction(num, den))


def target(alpha_star):
    """alpha_star to 2^-32: nearest integer to 2^32 alpha_star, ties to even."""
    return round(math.ldexp(float(alpha_star), 32))


def qualifies(E, dbeta, A):
    num, den = overlap_fraction(E, dbeta)
    return num * 2 ** 32 >= A * den


def step_rule(E, alpha_star, dbeta_max, iterations=60):
    """Largest dbeta in [0, dbeta_max] with alpha(dbeta) >= alpha_star (bisection)."""
    A = target(alpha_star)
    if qualifies(E, dbeta_max, A):
        return float(dbeta_max)
    lo, hi = 0.0, float(dbeta_max)
    for _ in range(iterations):
        mid = 0.5 * (lo + hi)
        if qualifies(E, mid, A):
            lo = mid
        else:
            hi = mid
    return lo


def learned_step(E, cand, alpha_star, dbeta_max, iterations=60, bracket=1.0, refine=0):
    """The learned step's exact check of a proposal (reading of the adaptive
    step with a learned proposal; the rule stays the arbiter).

    c = min(cand, dbeta_max).  refine = 0: c if alpha(c) >= alpha_star.
    refine > 0: if c qualifies, the top of [c, min(bracket c, dbeta_max)] if
    it qualifies, else that interval halved `refine` times keeping the lower
    end qualified; if c fails but c / bracket qualifies, [c / bracket, c]
    halved `refine` times.  Otherwise (or c <= 0) the rule decides.
    Returns (dbeta, fallback)."""
    A = target(alpha_star)
    c = min(float(cand), float(dbeta_max))
    if c > 0.0:
        ok = qualifies(E, c, A)
        if ok and (refine == 0 or c >= dbeta_max):
            return c, False
        if refine > 0:
            if ok:
                lo, hi = c, min(bracket * c, float(dbeta_max))
                if qualifies(E, hi, A):
                    return hi, False
                inside = True
            else:
                lo, hi = c / bracket, c
                inside = qualifies(E, lo, A)
            if inside:
                for _ in range(refine):
                    mid = 0.5 * (lo + hi)
                    if qualifies(E, mid, A):
                        lo = mid
                    else:
                        hi = mid
                return lo, False
    return step_rule(E, alpha_star, dbeta_max, iterations), True
