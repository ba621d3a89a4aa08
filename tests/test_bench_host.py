"""CPU checks of the benchmark's host-side accounting: interval unions, the
algorithmic byte count of a resampling, the code-only source key of the
counter profile, and the refusal of more than one GPU."""
import os
import subprocess
import sys

from tests.conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_union_of_intervals():
    assert bench.union_length([]) == 0.0
    assert bench.union_length([(0, 1), (2, 3)]) == 2
    assert bench.union_length([(0, 2), (1, 3)]) == 3
    assert bench.union_length([(1, 3), (0, 2), (5, 6), (2.5, 4)]) == 5
    assert bench.union_length([(0, 10), (1, 2), (3, 4)]) == 10


def test_resample_and_sweep_bytes():
    N = bench.L ** bench.D
    # 20 B per old replica; per new replica its spins read and written and 28 B
    assert bench.resample_bytes(N, 0, 0) == 0
    assert bench.resample_bytes(N, 10, 0) == 200
    assert bench.resample_bytes(N, 0, 3) == 3 * (2 * N / 8 + 28)
    # a sweep launch reads and writes each column once, and writes E and M
    assert bench.sweep_bytes(4096, 1) == 2 * 4096 * 8 + 64 * 8
    assert bench.sweep_bytes(4096, 15625) == 15625 * bench.sweep_bytes(4096, 1)


def test_headline_is_the_largest_single_run_configuration():
    # 3D +-J L = 16, R = 10^6, theta = 10, beta 0 -> 3 in 301 points, systematic
    assert (bench.D, bench.L, bench.R, bench.THETA, bench.BETA_F, bench.POINTS) == (3, 16, 10 ** 6, 10, 3.0, 301)
    assert bench.SCHEME == 3
    s = bench.schedule()
    assert s[0] == 0.0 and s[-1] == 3.0 and len(s) == 301


def test_roofline_fraction_is_the_philox_bound_fraction():
    """frac = (attempts / launch time) / (Philox rate / calls per attempt), which
    is the sweep's Philox call rate over the probe's."""
    attempts, calls, updates, words = 4.096e10, 2.0e9, 6.4e8, 15625
    r = bench.sweep_roofline("k", 4096, attempts, calls, updates, words, [2.0, 2.0], 1.0e12, "3d_pmj", None)
    cpa = calls / (64 * updates)
    assert abs(r["achieved"] - attempts / 4e-3 / 1e9) < 1e-6
    assert abs(r["peak"] - 1.0e12 / cpa / 1e9) < 1e-6
    assert abs(r["frac"] - (calls / 4e-3) / 1.0e12) < 1e-12
    assert r["bound"] == "alu" and r["unit"] == "attempts/ns" and r["traffic"] is None
    assert abs(r["hbm"]["achieved"] - 2 * bench.sweep_bytes(4096, words / 2) / 4e-3 / 1e9) < 1e-6


def test_profile_key_ignores_comments_only():
    a = "int f(int x) { return x + 1; } // one\n/* two\n three */ int g;"
    b = "int f(int x)\n{\n    return x + 1;   /* other words */\n}\nint g;"
    c = "int f(int x) { return x + 2; } int g;"
    assert bench.code_only(a) == bench.code_only(b)
    assert bench.code_only(a) != bench.code_only(c)
    assert len(bench.kernel_source_hash()) == 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)

