"""Pins of the weighted combination of runs, Eqs. (9)-(12) (CPU only)."""
import math

import numpy as np

from oracle.combine import combine


def run(R, lnZ, e=-1.0, e2=1.1, am=0.5, m2=0.3, beta=0.5):
    return dict(R=R, lnZ=lnZ, e=e, e2=e2, abs_m=am, m2=m2, beta=beta)


def test_equal_runs_give_the_plain_average():
    rs = [run(1000, 50.0, e=-1 - 0.1 * k) for k in range(5)]
    c = combine(rs, 64)
    assert abs(c["e"] - np.mean([r["e"] for r in rs])) < 1e-15
    assert abs(c["n_eff"] - 5) < 1e-12
    assert abs(c["lnZ"] - 50.0) < 1e-12


def test_weights_follow_eq10():
    rs = [run(1000, 10.0), run(2000, 11.0), run(500, 9.5)]
    c = combine(rs, 16)
    raw = [r["R"] * math.exp(r["lnZ"]) for r in rs]
    for o, x in zip(c["omega"], raw):
        assert abs(o - x / sum(raw)) < 1e-14
    assert abs(c["lnZ"] - math.log(sum(raw) / 3500)) < 1e-12


def test_shift_invariance_and_dominance():
    rs = [run(100, 1e4 + k, e=-k) for k in range(4)]
    c1 = combine(rs, 8)
    c2 = combine([dict(r, lnZ=r["lnZ"] - 1e4) for r in rs], 8)
    assert abs(c1["e"] - c2["e"]) < 1e-14 and abs((c1["lnZ"] - 1e4) - c2["lnZ"]) < 1e-9
    d = combine([run(100, 0.0, e=-1.0), run(100, 80.0, e=-2.0)], 8)
    assert abs(d["e"] + 2.0) < 1e-12 and abs(d["n_eff"] - 1) < 1e-12


def test_variance_estimators_eq11_eq12():
    # one run: c = beta^2 N (<e^2> - <e>^2), chi = beta N (<m^2> - <|m|>^2)
    c = combine([run(10, 0.0, e=-1.2, e2=1.5, am=0.4, m2=0.2, beta=0.7)], 100)
    assert abs(c["c"] - 0.49 * 100 * (1.5 - 1.44)) < 1e-12
    assert abs(c["chi"] - 0.7 * 100 * (0.2 - 0.16)) < 1e-12


def test_naive_and_plain_schemes():
    """W_var c exceeds the naive weighted c by exactly beta^2 N times the weighted
    variance of the runs' energies (and likewise for chi with |m|); identical
    runs make all schemes agree; equal weights make plain = weighted."""
    rs = [run(1000, 10.0, e=-1.0, e2=1.10, am=0.50, m2=0.30),
          run(2000, 11.0, e=-1.2, e2=1.50, am=0.40, m2=0.20),
          run(500, 9.5, e=-0.9, e2=0.85, am=0.60, m2=0.40)]
    N, b = 16, 0.5
    c = combine(rs, N)
    om = c["omega"]
    var_e = sum(o * (r["e"] - c["e"]) ** 2 for o, r in zip(om, rs))
    var_m = sum(o * (r["abs_m"] - c["abs_m"]) ** 2 for o, r in zip(om, rs))
    assert abs((c["c"] - c["c_naive"]) - b * b * N * var_e) < 1e-12
    assert abs((c["chi"] - c["chi_naive"]) - b * N * var_m) < 1e-12
    assert c["c"] >= c["c_naive"] and c["chi"] >= c["chi_naive"]
    same = combine([run(1000, 5.0 + k, e=-1.1, e2=1.3) for k in range(4)], N)
    assert abs(same["c"] - same["c_naive"]) < 1e-12 and abs(same["c_plain"] - same["c"]) < 1e-12
    eq = combine([run(700, 3.0, e=-1 - 0.1 * k, e2=1.2 + 0.05 * k) for k in range(5)], N)
    assert abs(eq["e_plain"] - eq["e"]) < 1e-15 and abs(eq["c_plain"] - eq["c_naive"]) < 1e-12
