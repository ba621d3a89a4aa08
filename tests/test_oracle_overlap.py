"""Pins of the oracle's overlap histogram (Figs. 6-7): against the direct
definition q = (1/N) sum_s sigma^a_s sigma^b_s on unpacked int8 spins,
and its special cases (a population against itself: every pair at q = 1;
against its negation: q = -1; independent random states: the binomial law's
mean and variance)."""
import numpy as np

from oracle import oracle as O


def pack(spins):
    """int8 spins [R][N] -> packed words [W][N] (bit b of word w = replica 64w + b, 1 for -1)."""
    R, N = spins.shape
    W = (R + 63) // 64
    bits = np.zeros((W * 64, N), np.uint64)
    bits[:R] = (spins < 0).astype(np.uint64)
    out = np.zeros((W, N), np.uint64)
    for b in range(64):
        out |= bits[b::64][:W] << np.uint64(b)
    return out


def test_matches_the_direct_definition_ragged():
    rng = np.random.default_rng(3)
    N = 27
    for Ra, Rb in ((200, 130), (64, 64), (65, 300), (1, 5)):
        a = np.where(rng.random((Ra, N)) < 0.3, -1, 1).astype(np.int8)
        b = np.where(rng.random((Rb, N)) < 0.6, -1, 1).astype(np.int8)
        R = min(Ra, Rb)
        q = (a[:R].astype(np.int64) * b[:R]).sum(axis=1)  # = 2k - N
        ref = np.bincount((q + N) // 2, minlength=N + 1)
        got = O.overlap_histogram(pack(a), pack(b), Ra, Rb, N)
        assert np.array_equal(got, ref)


def test_special_cases():
    rng = np.random.default_rng(5)
    N, R = 1000, 700
    a = np.where(rng.random((R, N)) < 0.5, -1, 1).astype(np.int8)
    h = O.overlap_histogram(pack(a), pack(a), R, R, N)
    assert h[N] == R and h.sum() == R
    h = O.overlap_histogram(pack(a), pack(-a), R, R, N)
    assert h[0] == R and h.sum() == R
    b = np.where(rng.random((R, N)) < 0.5, -1, 1).astype(np.int8)
    h = O.overlap_histogram(pack(a), pack(b), R, R, N)
    k = np.arange(N + 1)
    mean = (h * k).sum() / R
    var = (h * (k - mean) ** 2).sum() / R
    # k ~ Binomial(N, 1/2): mean N/2, variance N/4
    assert abs(mean - N / 2) < 5 * np.sqrt(N / 4 / R)
    assert 0.8 < var / (N / 4) < 1.2
