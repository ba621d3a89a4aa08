"""Pin of the oracle's ln Q (Eq. (1)) at the largest population, R = 2^24 - 64.

The oracle sums the R terms exp(-dbeta (E_j - E_min)) with Neumaier's
compensation.  Its ln Q is checked against the exact value written out
from the definition: the terms grouped by energy level (the sum over
replicas equals sum_levels n_E exp(-dbeta (E - E_min)) exactly), each level's
exponential and the logarithm evaluated in 50-digit mpmath.  The bound is
1e-14 of the larger of the two terms of ln Q = -dbeta E_min + ln(sum / R),
whose cancellation is what makes the sum's rounding matter.  The same terms
summed one after the other without compensation miss that bound at this R
(checked below), so a slip in the compensation that degrades it to a plain
sum fails the pin.  (Its other branch, for a term larger than the running
sum, only occurs while the running sum is below 1, before the first
lowest-level term, where the rounding it recovers is at most 2^-53 of the
total; no test of the sum at 1e-14 can see it.)"""
import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O

R = (1 << 24) - 64


def energies(seed, mean_u, sd_u, N=4096, d=2):
    """E = 2U - dN with U (unsatisfied bonds) spread around mean_u, in random order."""
    rng = np.random.default_rng(seed)
    U = np.clip(np.rint(rng.normal(mean_u, sd_u, R)), 0, d * N).astype(np.int64)
    return (2 * U - d * N).astype(np.int32)


def exact_lnQ(E, dbeta):
    levels, counts = np.unique(E, return_counts=True)
    emin = int(levels[0])
    with mp.workdps(50):
        db = mp.mpf(dbeta)
        s = mp.fsum(mp.mpf(int(c)) * mp.exp(-db * (int(e) - emin)) for e, c in zip(levels, counts))
        return -db * emin + mp.log(s / R), -db * emin, mp.log(s / R)


@pytest.mark.parametrize("seed,mean_u,sd_u,dbeta", [(1, 3000, 60, 0.003), (2, 1200, 25, 0.02),
                                                    (3, 600, 4, 0.05)])
def test_lnQ_at_the_largest_population(seed, mean_u, sd_u, dbeta):
    E = energies(seed, mean_u, sd_u)
    lnq, W, S = O.reweight(E, dbeta)
    ex, t1, t2 = exact_lnQ(E, dbeta)
    scale = float(max(abs(t1), abs(t2)))
    assert abs(lnq - float(ex)) <= 1e-14 * scale, (lnq, float(ex), scale)
    # the integer weights of the same call: W = floor(2^40 pa_exp(...)), S their sum
    assert int(W.max()) == 1 << 40 and int(W.sum(dtype=np.uint64)) == S


def test_a_plain_sum_misses_the_bound():
    """The sensitivity of the pin: summing the same double terms in order
    without compensation misses 1e-14 here."""
    E = energies(1, 3000, 60)
    dbeta = 0.003
    emin = int(E.min())
    terms = np.exp(-dbeta * (E - emin).astype(np.float64))
    plain = float(np.cumsum(terms)[-1])  # sequential, as a plain loop
    lnq_plain = -dbeta * emin + np.log(plain / R)
    ex, t1, t2 = exact_lnQ(E, dbeta)
    scale = float(max(abs(t1), abs(t2)))
    assert abs(lnq_plain - float(ex)) > 1e-14 * scale
