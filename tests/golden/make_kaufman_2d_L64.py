"""Writes kaufman_2d_L64.json: exact values of the 2D periodic Ising
ferromagnet, L = 64, along the schedule beta_i = 0.6 i / 200 (every 20th
point and the last), from Kaufman's finite-torus partition function (the
oracle's exact module; the only code this script calls).

    python tests/golden/make_kaufman_2d_L64.py

Stored per point: ln Z (60-digit evaluation rounded to double), the energy
per spin e = <E>/N and the specific heat per spin c = beta^2 Var(E)/N (central
differences of ln Z).  The benchmark reads this file to report each
resampling scheme's free-energy error at the end of the anneal; it never
runs the oracle itself.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402

L, BETA_F, POINTS = 64, 0.6, 201


def main():
    rows = []
    for i in list(range(0, POINTS, 20)) + ([POINTS - 1] if (POINTS - 1) % 20 else []):
        beta = i * BETA_F / (POINTS - 1)
        e, c = exact.kaufman_e_c(L, beta) if beta > 0 else (0.0, 0.0)
        rows.append({"i": i, "beta": beta, "lnZ": exact.kaufman_lnZ(L, beta), "e": e, "c": c})
    out = {"system": "2D Ising ferromagnet, L = 64, periodic, J = 1",
           "schedule": "beta_i = 0.6 i / 200, i = 0..200",
           "source": "Kaufman, Phys. Rev. 76, 1232 (1949), finite-torus Z (four-term form of "
                     "Ferdinand & Fisher, Phys. Rev. 185, 832 (1969)), 60 digits",
           "points": rows}
    with open(os.path.join(HERE, "kaufman_2d_L64.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
