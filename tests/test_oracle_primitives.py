"""Pins of the oracle's primitives: Philox4x32-10, the deterministic exp and the
Metropolis thresholds (CPU only)."""
import math
import os
import shutil
import subprocess
import tempfile

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch_include():
    try:
        import torch.utils.cpp_extension as ce
        for p in ce.include_paths():
            if os.path.exists(os.path.join(p, "ATen", "core", "PhiloxRNGEngine.h")):
                return p
    except Exception:
        pass
    return None


@pytest.fixture(scope="module")
def torch_philox():
    inc = _torch_include()
    if inc is None or shutil.which("g++") is None:
        pytest.skip("torch headers or g++ missing")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_ref")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", inc,
                    os.path.join(HERE, "philox_torch_ref.cpp"), "-o", exe], check=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_independent_engine(torch_philox):
    """Philox4x32-10 (Salmon et al., SC'11) against PyTorch's own engine."""
    rng = np.random.default_rng(12345)
    cases = rng.integers(0, 2 ** 32, size=(500, 6), dtype=np.uint64)
    cases[0] = 0
    cases[1] = 2 ** 32 - 1
    cases[2, 2:] = [3, 0, 7, (2 << 28) | (5 << 8) | 15]  # a METRO-shaped counter
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in cases) + "\n"
    out = subprocess.run([torch_philox], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for row, line in zip(cases, out):
        ref = [int(v) for v in line.split()]
        got = O.philox(int(row[0]), int(row[1]), [int(v) for v in row[2:]]).tolist()
        assert got == ref, (row, got, ref)


def test_philox_changes_with_every_counter_and_key_word():
    base = O.philox(1, 0, [0, 0, 0, 0])
    for k in range(4):
        ctr = [0, 0, 0, 0]
        ctr[k] = 1
        assert not np.array_equal(O.philox(1, 0, ctr), base)
    assert not np.array_equal(O.philox(2, 0, [0, 0, 0, 0]), base)
    assert not np.array_equal(O.philox(1, 1, [0, 0, 0, 0]), base)


def _ulp_err(x):
    got = O.pa_exp(x)
    with mp.workdps(40):
        ref = mp.exp(mp.mpf(x))
        ulp = math.ulp(float(ref))
        return float(abs(mp.mpf(got) - ref) / ulp)


def test_pa_exp_error_bound():
    """The decision exp is within 1.5 ulp of exp on [-700, 0] (mpmath reference)."""
    rng = np.random.default_rng(7)
    xs = list(-700.0 * rng.random(3000)) + list(-rng.random(3000)) + list(-1e-3 * rng.random(500))
    xs += [-math.log(2.0) * k for k in range(1, 60)] + [-0.5 * math.log(2.0), -1e-300, -700.0]
    worst = max(_ulp_err(x) for x in xs)
    assert worst <= 1.5, worst


def test_pa_exp_special_values():
    assert O.pa_exp(0.0) == 1.0
    assert O.pa_exp(-0.0) == 1.0
    assert O.pa_exp(-700.5) == 0.0
    assert O.pa_exp(float("nan")) == 0.0
    # exp(-k ln 2) is a power of two up to the rounding of its argument
    for k in range(1, 40):
        assert abs(O.pa_exp(-k * math.log(2.0)) * 2.0 ** k - 1.0) < 1e-14


def test_metropolis_threshold():
    # beta = 0 accepts everything: T = 2^32 exceeds every 32-bit uniform
    for dE in (4, 8, 12):
        assert O.threshold(0.0, dE) == 2 ** 32
    for beta in (0.1, 0.44068, 1.0, 3.0):
        prev = 2 ** 32
        for dE in (4, 8, 12):
            T = O.threshold(beta, dE)
            ref = 2.0 ** 32 * math.exp(-beta * dE)
            assert abs(T - ref) <= 1.0
            assert T <= prev
            prev = T
    assert O.threshold(100.0, 4) == 0
