"""Oracle of the free-energy-weighted combination of runs (Sec. 4), test
infrastructure only.

Eq. (7) gives each run m a free-energy estimate, ln Z_hat^(m) = -beta F_hat^(m)
(relative to Z_0); Eq. (10) weights its estimates by
omega_m = R^(m) exp(-beta F_hat^(m)) / sum_m R^(m) exp(-beta F_hat^(m)), and
Eq. (9) forms W[O] = sum_m omega_m O^(m).  Variances are weighted through
their non-central moments, Eqs. (11)-(12); for comparison (the left column of
Fig. 5 and the plain averages of Fig. 8) also the naive weighted averages of
the runs' own c and chi, and the plain unweighted means over the runs.  For a
fluctuating population size
R^(m) is the run's size at the point (reading: the paper calls the exact
expression "a bit more complicated").  Computed in log space against the
largest l_m = ln R^(m) + ln Z_hat^(m).
"""
import math


def combine(runs, N):
    """runs: dicts with R, lnZ, beta, e, e2, abs_m, m2 (per-spin averages)."""
    l = [math.log(r["R"]) + r["lnZ"] for r in runs]
    lmax = max(l)
    w = [math.exp(x - lmax) for x in l]
    den = sum(w)
    om = [x / den for x in w]
    Rsum = sum(r["R"] for r in runs)
    W = {k: sum(o * r[k] for o, r in zip(om, runs)) for k in ("e", "e2", "abs_m", "m2")}
    beta = runs[0]["beta"]
    # each run's own variance estimates
    c_m = [beta * beta * N * (r["e2"] - r["e"] ** 2) for r in runs]
    chi_m = [beta * N * (r["m2"] - r["abs_m"] ** 2) for r in runs]
    M = len(runs)
    return dict(lnZ=lmax + math.log(den) - math.log(Rsum), e=W["e"], e2=W["e2"],
                abs_m=W["abs_m"], m2=W["m2"], c=beta * beta * N * (W["e2"] - W["e"] ** 2),
                chi=beta * N * (W["m2"] - W["abs_m"] ** 2), n_eff=1.0 / sum(o * o for o in om),
                runs=M, beta=beta, omega=om,
                c_naive=sum(o * x for o, x in zip(om, c_m)),
                chi_naive=sum(o * x for o, x in zip(om, chi_m)),
                e_plain=sum(r["e"] for r in runs) / M, c_plain=sum(c_m) / M, chi_plain=sum(chi_m) / M)
