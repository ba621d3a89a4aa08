"""A temperature step of the single-run calls, deferred, captured into a HIP
graph (through torch's graph capture on the run's own stream) and replayed:
every replay must give the bits the same step gives when issued eagerly.  The
captured step reweights to a fixed beta, so replays after the first are steps
of zero width; the Philox counters still advance with the device-side step
index."""
import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scheme", [O.NEAREST_INT, O.SYSTEMATIC])
def test_captured_step_replays_match_eager_steps(scheme):
    import torch
    from paper_2401_07965_amd import pa
    d, L, R, theta = 2, 16, 3000, 4
    print(f"[graph] capture one step, scheme={scheme}", flush=True)
    s = torch.cuda.Stream()
    a = pa.PARun(d, L, R, seed=4, run_id=scheme, stream=s)
    b = pa.PARun(d, L, R, seed=4, run_id=scheme)
    warm = (0.05, 0.1)
    for beta in warm:
        for g in (a, b):
            g.reweight(beta, wait=False)
            g.resample(scheme, wait=False)
            g.sweep(theta)
            g.observables(wait=False)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        a.reweight(0.3, wait=False)
        a.resample(scheme, wait=False)
        a.sweep(theta)
        a.observables(wait=False)
    for k in range(4):
        graph.replay()
        torch.cuda.synchronize()  # eager work of the program between replays
        b.reweight(0.3, wait=False)
        b.resample(scheme, wait=False)
        b.sweep(theta)
        b.observables(wait=False)
        sa, sb = a.export(), b.export()
        for key in ("spins", "energy", "magnetization", "label"):
            assert np.array_equal(sa[key], sb[key]), (k, key)
        assert sa["R"] == sb["R"] and sa["lnZ"] == sb["lnZ"] and sa["step"] == sb["step"] == 3 + k
        assert a.observables() == b.observables()
    del graph
    a.close()
    b.close()
