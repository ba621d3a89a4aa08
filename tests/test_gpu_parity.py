"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the
same seeded inputs.  Spins, energies, magnetisations, labels, population
sizes and the exact integer sums must be bit-identical; ln Q, ln Z_hat and the
finalised averages agree to 1e-10 relative."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests.paritylib import (compare_state, ea_couplings, rel_ok, run_pair, sampled_step,
                             schedule)

pytestmark = pytest.mark.gpu

SCHEMES = [O.MULTINOMIAL, O.POISSON, O.NEAREST_INT, O.SYSTEMATIC]


def test_2d_L8_R1000_every_step():
    """2D Ising FM, L = 8, R = 1000, beta 0 -> 1 in 101 points, theta = 10, nearest integer."""
    g, o = run_pair(2, 8, 1000, O.NEAREST_INT, schedule(1.0, 101), 10, seed=1, run_id=0)
    assert rel_ok(g.free_energy(), o.free_energy())
    g.close()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_schemes_2d_ragged(scheme):
    g, _ = run_pair(2, 8, 300, scheme, schedule(1.2, 21), 5, seed=7, run_id=scheme)
    g.close()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_schemes_3d_spin_glass(scheme):
    J = ea_couplings(3, 4, 3)
    g, _ = run_pair(3, 4, 200, scheme, schedule(2.0, 16), 3, seed=2, run_id=10 + scheme, J=J)
    g.close()


@pytest.mark.parametrize("d,L,R", [(2, 6, 130), (2, 2, 70), (3, 2, 70), (2, 4, 1), (2, 4, 64),
                                   (2, 4, 65), (3, 6, 129)])
def test_shapes_and_edge_sizes(d, L, R):
    J = ea_couplings(d, L, 5)
    for scheme in (O.SYSTEMATIC, O.NEAREST_INT):
        g, _ = run_pair(d, L, R, scheme, schedule(1.5, 9), 2, seed=3, run_id=scheme, J=J)
        g.close()


@pytest.mark.parametrize("d,L,kind,R,scheme", [(2, 128, "fm", 130, O.NEAREST_INT),
                                                (2, 128, "ea", 65, O.POISSON),
                                                (3, 24, "ea", 70, O.SYSTEMATIC),
                                                (3, 24, "fm", 64, O.MULTINOMIAL)])
def test_largest_lattices(d, L, kind, R, scheme):
    """The largest lattices one workgroup holds in LDS: N = 16384 (2D L = 128)
    and 13824 (3D L = 24), with and without couplings."""
    J = ea_couplings(d, L, 17) if kind == "ea" else None
    g, _ = run_pair(d, L, R, scheme, schedule(1.0, 4), 2, seed=4, run_id=scheme, J=J)
    g.close()


def test_large_steps_and_poisson_pieces():
    # few, large steps: broad weights, tauhat > 32 for the lowest energies
    for scheme in SCHEMES:
        g, _ = run_pair(2, 8, 400, scheme, [0.0, 0.5, 1.5, 3.0], 2, seed=4, run_id=scheme,
                        capacity=4096)
        g.close()


def test_zero_step_and_zero_sweeps():
    from paper_2401_07965_amd import pa
    g = pa.PARun(2, 6, 100, seed=9, capacity=256)
    o = O.OracleRun(2, 6, 100, seed=9, capacity=256)
    for b in (0.0, 0.0, 0.3, 0.3):
        qg, qo = g.reweight(b), o.reweight(b)
        assert rel_ok(qg, qo)
        assert g.resample(O.SYSTEMATIC) == o.resample(O.SYSTEMATIC)
        g.sweep(0)
        compare_state(g, o)
    g.close()


def test_capacity_and_extinction_leave_state_unchanged():
    from paper_2401_07965_amd import pa
    g = pa.PARun(2, 4, 64, seed=5, capacity=64)
    o = O.OracleRun(2, 4, 64, seed=5, capacity=64)
    g.reweight(0.0)
    o.reweight(0.0)
    before = g.export()
    raised = False
    for step in range(30):
        b = 0.5 * (step + 1)
        g.reweight(b)
        o.reweight(b)
        try:
            rg = g.resample(O.POISSON)
        except pa.CapacityError:
            with pytest.raises(O.CapacityError):
                o.resample(O.POISSON)
            raised = True
            break
        assert rg == o.resample(O.POISSON)
        before = g.export()
    assert raised
    after = g.export()
    for k in ("spins", "energy", "label", "magnetization"):
        assert np.array_equal(before[k], after[k])
    assert before["lnZ"] == after["lnZ"] and before["beta"] == after["beta"]
    g.close()


def test_call_order_and_argument_errors():
    from paper_2401_07965_amd import pa
    g = pa.PARun(2, 4, 10, seed=1)
    with pytest.raises(pa.StateError):
        g.resample(O.SYSTEMATIC)
    g.reweight(0.5)
    g.reweight(0.1)  # a second reweight replaces the first
    g.resample(O.SYSTEMATIC)
    with pytest.raises(pa.PAError):
        g.reweight(0.05)  # beta must not decrease
    with pytest.raises(pa.PAError):
        g.reweight(float("nan"))
    with pytest.raises(pa.PAError):
        g.sweep(-1)
    g.close()
    for bad in (dict(dim=4, L=4, R=10), dict(dim=2, L=5, R=10), dict(dim=2, L=4, R=0),
                dict(dim=2, L=4, R=100, capacity=50), dict(dim=3, L=32, R=10)):
        with pytest.raises(pa.PAError):
            pa.pa_required_bytes(pa.make_config(**bad))


def test_export_import_roundtrip_continues_identically():
    from paper_2401_07965_amd import pa
    J = ea_couplings(2, 6, 8)
    betas = schedule(1.0, 11)
    g, o = run_pair(2, 6, 150, O.NEAREST_INT, betas[:6], 3, seed=6, J=J, observables=False)
    st = g.export()
    h = pa.PARun(2, 6, 150, seed=6, couplings=J)
    h.import_state(R=st["R"], step=st["step"], sweeps=st["sweeps"], beta=st["beta"],
                   lnZ=st["lnZ"], spins=st["spins"], energy=st["energy"],
                   magnetization=st["magnetization"], label=st["label"])
    for b in betas[6:]:
        assert g.reweight(b) == h.reweight(b)
        assert g.resample(O.NEAREST_INT) == h.resample(O.NEAREST_INT)
        g.sweep(3)
        h.sweep(3)
    a, c = g.export(), h.export()
    for k in ("spins", "energy", "magnetization", "label"):
        assert np.array_equal(a[k], c[k])
    assert a["lnZ"] == c["lnZ"]
    # an oracle state imported into the GPU continues like the oracle
    h.import_state(R=o.Rcur, step=o.step, sweeps=o.t, beta=o.beta, lnZ=o.free_energy(),
                   spins=pa.pack_spins(o.spins), energy=o.E,
                   magnetization=o.magnetization().astype(np.int32), label=o.label)
    for b in betas[6:]:
        assert rel_ok(h.reweight(b), o.reweight(b))
        assert h.resample(O.SYSTEMATIC) == o.resample(O.SYSTEMATIC)
        h.sweep(3)
        o.sweep(3)
    compare_state(h, o)
    g.close()
    h.close()


def test_repeat_runs_are_bit_identical():
    """Any race in the kernels would flip a bit between two identical runs."""
    from paper_2401_07965_amd import pa
    out = []
    for _ in range(2):
        g = pa.PARun(2, 16, 3000, seed=11, run_id=2)
        for b in schedule(0.8, 9)[1:]:
            g.reweight(b)
            g.resample(O.MULTINOMIAL)
            g.sweep(4)
        out.append((g.export(), g.observables()))
        g.close()
    for k in ("spins", "energy", "magnetization", "label"):
        assert np.array_equal(out[0][0][k], out[1][0][k])
    assert out[0][0]["lnZ"] == out[1][0]["lnZ"]
    assert out[0][1] == out[1][1]


@pytest.mark.parametrize("d,L", [(3, 4), (3, 10), (2, 32)])
def test_overlap_distribution(d, L):
    """P(q) of two populations of the same couplings: N = 64 (one site per
    thread), 1000 (three or four sites per thread, the last pair ragged) and
    1024 (four)."""
    J = ea_couplings(d, L, 12)
    betas = schedule(1.0, 6)
    print(f"[parity] overlap d={d} L={L}", flush=True)
    ga, oa = run_pair(d, L, 300, O.SYSTEMATIC, betas, 2, seed=1, run_id=0, J=J,
                      observables=False)
    gb, ob = run_pair(d, L, 250, O.NEAREST_INT, betas, 2, seed=1, run_id=1, J=J,
                      observables=False)
    h = ga.overlap(gb)
    R = min(oa.Rcur, ob.Rcur)
    N = L ** d
    same = (oa.spins[:R] == ob.spins[:R]).sum(axis=1)  # N - popcount(a ^ b)
    ref = np.bincount(same, minlength=N + 1)
    assert np.array_equal(h, ref)
    ga.close()
    gb.close()


def test_2d_L64_R1e5_sampled_full_size():
    """2D Ising FM, L = 64, R = 10^5, theta = 10, beta_i = 0.6 i/200: sampled steps, all schemes."""
    from paper_2401_07965_amd import pa
    betas = schedule(0.6, 201)
    rng = np.random.default_rng(0)
    for scheme in SCHEMES:
        print(f"[parity] 2D L=64 R=1e5 sampled step, scheme {scheme}", flush=True)
        g = pa.PARun(2, 64, 100000, seed=1, run_id=scheme)
        for i in range(1, 4):
            g.reweight(betas[i])
            g.resample(scheme)
            g.sweep(10)
        rows = np.concatenate([np.arange(64), np.arange(99936, 100000),
                               rng.integers(0, 99000, 64)])
        sampled_step(g, 2, 64, None, scheme, betas[4], 10, rows, 1, scheme, 100000)
        g.close()


def test_3d_L10_R5e5_sampled_full_size():
    """3D +-J glass, L = 10, R = 5 10^5, systematic, theta = 10, beta_i = 3 i/300: sampled step."""
    from paper_2401_07965_amd import pa
    J = ea_couplings(3, 10, 1)
    betas = schedule(3.0, 301)
    g = pa.PARun(3, 10, 500000, seed=1, run_id=0, couplings=J)
    for i in range(1, 3):
        g.reweight(betas[i])
        g.resample(O.SYSTEMATIC)
        g.sweep(10)
    rows = np.concatenate([np.arange(64), np.arange(499900, 500000),
                           np.random.default_rng(1).integers(0, 499000, 64)])
    sampled_step(g, 3, 10, J, O.SYSTEMATIC, betas[3], 10, rows, 1, 0, 500000)
    g.close()


def test_3d_L16_R1e6_sampled_full_size():
    """3D +-J glass, L = 16, R = 10^6 (the learned-schedule workload's size and
    the sweep's fixed-axis walk in 3D), systematic, theta = 10: sampled step."""
    from paper_2401_07965_amd import pa
    J = ea_couplings(3, 16, 1)
    print("[parity] 3D L=16 R=1e6 sampled step", flush=True)
    g = pa.PARun(3, 16, 1000000, seed=1, run_id=0, couplings=J)
    for b in (0.01, 0.02):
        g.reweight(b)
        g.resample(O.SYSTEMATIC)
        g.sweep(10)
    rows = np.concatenate([np.arange(64), np.arange(999936, 1000000),
                           np.random.default_rng(2).integers(0, 999000, 64)])
    sampled_step(g, 3, 16, J, O.SYSTEMATIC, 0.03, 10, rows, 1, 0, 1000000)
    g.close()


def test_philox_probe_matches_the_oracle_generator():
    """The throughput probe evaluates the same generator as the sweeps."""
    import torch
    from paper_2401_07965_amd import pa
    out = torch.empty(1024, dtype=torch.int32, device="cuda")
    pa.philox_probe(out, 3, torch.cuda.current_stream())
    got = out.cpu().numpy().view(np.uint32)
    for t in (0, 1, 255, 700, 1023):
        acc = 0
        for i in range(3):
            for q in range(3):
                x = O.philox(1, 2, [t, i, 7, (2 << 28) | q])
                acc ^= int(x[0]) ^ int(x[1]) ^ int(x[2]) ^ int(x[3])
        assert int(got[t]) == acc, t


def test_extinction_matches_oracle_and_leaves_the_state():
    """One replica, Poisson resampling: the step that would empty the
    population fails on both sides at the same step, state unchanged."""
    from paper_2401_07965_amd import pa
    g = pa.PARun(2, 4, 1, seed=2, run_id=1)
    o = O.OracleRun(2, 4, 1, seed=2, run_id=1)
    for s in range(40):
        b = 0.01 * (s + 1)
        assert rel_ok(g.reweight(b), o.reweight(b))
        before = g.export()
        try:
            o.resample(O.POISSON)
        except O.ExtinctError:
            with pytest.raises(pa.ExtinctError):
                g.resample(O.POISSON)
            after = g.export()
            for k in ("spins", "energy", "label", "magnetization"):
                assert np.array_equal(before[k], after[k])
            assert before["lnZ"] == after["lnZ"] and before["R"] == after["R"] == 1
            break
        assert g.resample(O.POISSON) == o.Rcur
        g.sweep(1)
        o.sweep(1)
        compare_state(g, o, f"step {s}")
    else:
        raise AssertionError("no extinction in 40 steps")
    g.close()


@pytest.mark.parametrize("d,L,R,scheme,J,beta_f", [(2, 8, 640, O.SYSTEMATIC, None, 1.2),
                                                   (3, 4, 256, O.MULTINOMIAL, "glass", 1.2),
                                                   (2, 16, 640, O.SYSTEMATIC, None, 1.2),
                                                   (3, 16, 128, O.SYSTEMATIC, "glass", 2.6)])
def test_work_counters_match_the_oracle_count(d, L, R, scheme, J, beta_f):
    """The sweeps' Philox count (the roofline's work figure) equals the oracle's
    count of plane pairs the decisions need, and the site and attempt counts
    their closed forms (full 64-replica words, fixed-size resampling).  The
    ordered ferromagnet and the glass at beta = 2.6 leave most sites with no
    replica to decide, so within a wave some lanes need pairs and others
    none (the 3D L = 16 case takes the fixed-axis walk with wave-uniform z
    offsets)."""
    from paper_2401_07965_amd import pa
    Jc = ea_couplings(d, L, 3) if J else None
    print(f"[parity] work counters d={d} L={L} R={R} scheme={scheme} beta_f={beta_f}", flush=True)
    g = pa.PARun(d, L, R, seed=6, run_id=1, couplings=Jc)
    o = O.OracleRun(d, L, R, seed=6, run_id=1, J=Jc)
    theta, steps = 4, 12
    for beta in schedule(beta_f, steps + 1)[1:]:
        g.reweight(beta)
        o.reweight(beta)
        g.resample(scheme)
        o.resample(scheme)
        g.sweep(theta)
        o.sweep(theta)
    c = g.counters()
    assert c["philox_calls"] == o.philox_calls > 0
    assert c["site_updates"] == steps * theta * L ** d * (R // 64)
    assert c["spin_attempts"] == steps * theta * L ** d * R
    compare_state(g, o, f"work counters d={d} L={L}")
    g.close()


def test_largest_population():
    """R = capacity = 2^24 - 64 on a 4x4 lattice: weight sums reach ~2^64 (the
    scan's inclusive prefixes outgrow its 62-bit tile words and later tiles add
    aggregates instead), 2048 scan tiles, and the 128-bit copy-number
    arithmetic at its bound; systematic and multinomial steps against the
    oracle, whole population."""
    from paper_2401_07965_amd import pa
    d, L, R = 2, 4, (1 << 24) - 64
    print(f"[parity] largest population d={d} L={L} R={R}", flush=True)
    g = pa.PARun(d, L, R, seed=2, run_id=0, capacity=R)
    o = O.OracleRun(d, L, R, seed=2, run_id=0, capacity=R)
    for beta, scheme in ((0.004, O.SYSTEMATIC), (0.008, O.MULTINOMIAL), (0.05, O.SYSTEMATIC)):
        qg, qo = g.reweight(beta), o.reweight(beta)
        assert rel_ok(qg, qo), (qg, qo)
        assert g.resample(scheme) == o.resample(scheme) == R
        g.sweep(1)
        o.sweep(1)
    assert o.pending is None and o.last_counts is not None
    compare_state(g, o, "largest population")
    g.close()


def test_largest_population_nearest_and_poisson():
    """Nearest-integer and Poisson resampling at R = 2^24 - 64 - 2^14 on a 4x4
    lattice (capacity 2^24 - 64): the copy numbers are drawn and summed in one
    pass over 4096-slot tiles (4096 tiles) with the 128-bit rounding test at
    its bound; sizes, a capacity failure if one occurs, and the whole
    population against the oracle; the sampling variance within 1e-9."""
    from paper_2401_07965_amd import pa
    d, L, cap = 2, 4, (1 << 24) - 64
    R = cap - (1 << 14)
    print(f"[parity] largest population, nearest and Poisson, R={R}", flush=True)
    g = pa.PARun(d, L, R, seed=3, run_id=1, capacity=cap)
    o = O.OracleRun(d, L, R, seed=3, run_id=1, capacity=cap)
    for beta, scheme in ((0.004, O.NEAREST_INT), (0.01, O.POISSON), (0.05, O.NEAREST_INT)):
        qg, qo = g.reweight(beta), o.reweight(beta)
        assert rel_ok(qg, qo), (qg, qo)
        try:
            rg = g.resample(scheme)
        except pa.CapacityError:
            with pytest.raises(O.CapacityError):
                o.resample(scheme)
            continue
        assert rg == o.resample(scheme), scheme
        sv = g.observables()["sv"]
        assert rel_ok(sv, o.last_sv, 1e-9) or abs(sv - o.last_sv) < 1e-14, (sv, o.last_sv)
        g.sweep(1)
        o.sweep(1)
    compare_state(g, o, "largest population, nearest and Poisson")
    g.close()


@pytest.mark.parametrize("d,L,R,glass", [(2, 8, 130, False), (2, 6, 70, True), (3, 4, 200, True)])
def test_sweeps_at_beta_zero_flip_every_spin(d, L, R, glass):
    """Sweeps right after the initial sampling run at beta = 0, where every
    energy-change class accepts outright (threshold 2^32): one sweep negates
    every spin, a second restores it, no random bits are drawn, and the
    energies are the oracle's."""
    from paper_2401_07965_amd import pa
    J = ea_couplings(d, L, 7) if glass else None
    print(f"[parity] sweeps at beta = 0, d={d} L={L} R={R} glass={glass}", flush=True)
    g = pa.PARun(d, L, R, seed=8, run_id=2, couplings=J)
    o = O.OracleRun(d, L, R, seed=8, run_id=2, J=J)
    start = compare_state(g, o, "initial")
    s0 = pa.unpack_spins(start["spins"], R)
    g.sweep(1)
    o.sweep(1)
    st = compare_state(g, o, "one sweep")
    assert np.array_equal(pa.unpack_spins(st["spins"], R), -s0)
    assert np.array_equal(st["energy"], start["energy"])  # E(-s) = E(s)
    g.sweep(1)
    o.sweep(1)
    st = compare_state(g, o, "two sweeps")
    assert np.array_equal(pa.unpack_spins(st["spins"], R), s0)
    assert g.counters()["philox_calls"] == 0 == o.philox_calls
    g.close()
