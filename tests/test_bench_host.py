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


def test_resample_bytes():
    N = bench.L ** bench.D
    # 20 B per old replica; per new replica its spins read and written and 28 B
    assert bench.resample_bytes(0, 0) == 0
    assert bench.resample_bytes(10, 0) == 200
    assert bench.resample_bytes(0, 3) == 3 * (2 * N / 8 + 28)


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

