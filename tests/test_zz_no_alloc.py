"""The allocation-free overlap entry point (pa_overlap_noalloc) through the C
ABI: the same histogram as pa_overlap, on two calls in a row, the second on
a smaller input (a smaller lattice and population), so that counters the
first call left in the shared device array must not leak into the second;
then the first input again, and the size and lattice checks."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from tests.paritylib import ea_couplings, schedule

pytestmark = pytest.mark.gpu


def annealed(d, L, R, run_id, J, betas):
    from paper_2401_07965_amd import pa
    g = pa.PARun(d, L, R, seed=3, run_id=run_id, couplings=J)
    for b in betas[1:]:
        g.reweight(b)
        g.resample(O.SYSTEMATIC)
        g.sweep(2)
    return g


def test_noalloc_overlap_equals_overlap_twice_then_smaller():
    from paper_2401_07965_amd import pa
    print("[no-alloc] 3D L=10 then 2D L=4", flush=True)
    betas = schedule(1.2, 7)
    J3 = ea_couplings(3, 10, 4)
    a, b = annealed(3, 10, 3000, 0, J3, betas), annealed(3, 10, 2500, 1, J3, betas)
    ref = a.overlap(b)
    got = a.overlap_noalloc(b)
    assert got.dtype == np.int64 and got.shape == (1001,)
    assert np.array_equal(got, ref) and got.sum() == 2500
    # second call, smaller: N = 16, 40 pairs
    J2 = ea_couplings(2, 4, 5)
    c, e = annealed(2, 4, 40, 0, J2, betas), annealed(2, 4, 70, 1, J2, betas)
    ref2 = c.overlap(e)
    got2 = c.overlap_noalloc(e)
    assert np.array_equal(got2, ref2) and got2.sum() == 40
    # and the first input once more
    assert np.array_equal(a.overlap_noalloc(b), ref)
    # different lattices: rejected before any launch
    with pytest.raises(pa.PAError):
        a.overlap_noalloc(c)
    lib = pa.lib()
    assert lib.pa_overlap_noalloc(a.ctx, b.ctx, None) == pa.PA_E_INVAL
    for g in (a, b, c, e):
        g.close()


def test_noalloc_overlap_at_the_largest_lattice():
    """N = 16384 (2D L = 128): all 16385 counters of the array in use."""
    from paper_2401_07965_amd import pa
    print("[no-alloc] 2D L=128", flush=True)
    betas = schedule(0.5, 3)
    a, b = annealed(2, 128, 200, 0, None, betas), annealed(2, 128, 130, 1, None, betas)
    ref = a.overlap(b)
    h = np.full(16385, -7, np.int64)
    st = pa.lib().pa_overlap_noalloc(a.ctx, b.ctx, h.ctypes.data_as(ctypes.c_void_p))
    assert st == pa.PA_OK
    assert np.array_equal(h, ref) and h.sum() == 130
    a.close()
    b.close()
