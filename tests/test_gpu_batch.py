"""GPU tests of batches: a batched anneal (eager or one HIP graph, any tuned
workgroup size) gives exactly the bits of the same runs done one by one
through the single-run calls; the weighted combination matches its oracle."""
import numpy as np
import pytest

from oracle import combine as OC
from oracle import oracle as O
from tests.paritylib import compare_state, ea_couplings, rel_ok, schedule

pytestmark = pytest.mark.gpu

SHAPES = [(2, 8, 300, "fm"), (3, 4, 200, "ea"), (2, 6, 130, "ea"), (3, 6, 500, "ea"),
          (2, 12, 1000, "fm"), (2, 8, 65, "ea"), (3, 4, 1, "fm"), (2, 16, 700, "ea")]


def configs(seed=3, single_replica=True):
    out = []
    for k, (d, L, R, kind) in enumerate(SHAPES):
        if R == 1 and not single_replica:
            continue
        J = None if kind == "fm" else ea_couplings(d, L, 100 + k)
        out.append(dict(dim=d, L=L, R=R, seed=seed, run_id=k, couplings=J))
    return out


def single_records(cfg, betas, theta, scheme):
    from paper_2401_07965_amd import pa
    g = pa.PARun(cfg["dim"], cfg["L"], cfg["R"], seed=cfg["seed"], run_id=cfg["run_id"],
                 couplings=cfg["couplings"])
    rows = []
    ob = g.observables()
    rows.append((0.0, g.free_energy(), ob))
    for b in betas[1:]:
        q = g.reweight(b)
        g.resample(scheme)
        g.sweep(theta)
        rows.append((q, g.free_energy(), g.observables()))
    st = g.export()
    g.close()
    return rows, st


@pytest.mark.parametrize("scheme", [O.SYSTEMATIC, O.NEAREST_INT, O.MULTINOMIAL, O.POISSON])
def test_batch_equals_single_runs(scheme):
    from paper_2401_07965_amd import pa
    betas = schedule(1.5, 9)
    # a one-replica Poisson run dies out with probability 1/e per step
    cfgs = configs(single_replica=scheme != O.POISSON)
    print(f"[batch] scheme {scheme}: {len(cfgs)} runs", flush=True)
    B = pa.PABatch(cfgs, max_points=len(betas))
    B.anneal(betas, 3, scheme, use_graph=False)
    rec = B.records()
    for m, cfg in enumerate(cfgs):
        rows, st = single_records(cfg, betas, 3, scheme)
        for i, (q, lz, ob) in enumerate(rows):
            r = rec[m, i]
            assert r["lnQ"] == q and r["lnZ"] == lz, (m, i)
            for k in ("e", "e2", "abs_m", "m2", "rho_t", "S_f", "sv"):
                assert r[k] == ob[k], (m, i, k)
            for k in ("R", "sum_E", "sum_E2", "sum_absM", "sum_M2", "sum_c2", "families"):
                assert int(r[k]) == int(ob[k]), (m, i, k)
        bs = B.export_run(m)
        for k in ("spins", "energy", "magnetization", "label"):
            assert np.array_equal(bs[k], st[k]), (m, k)
    B.close()


def test_graph_replays_equal_eager_and_tuning_changes_nothing():
    from paper_2401_07965_amd import pa
    betas = schedule(2.0, 12)
    B = pa.PABatch(configs(seed=5), max_points=len(betas))
    B.anneal(betas, 4, O.SYSTEMATIC, use_graph=False)
    ref = B.records().copy()
    ref_state = [B.export_run(m) for m in range(B.n)]
    threads = B.tune(4)
    assert all(t in (64, 128, 192, 256, 320, 384, 448, 512) for t in threads)
    for rep in range(3):
        print(f"[batch] graph replay {rep}", flush=True)
        B.anneal(betas, 4, O.SYSTEMATIC, use_graph=True)
        got = B.records()
        assert np.array_equal(got, ref), rep
        for m in range(B.n):
            s = B.export_run(m)
            for k in ("spins", "energy", "label"):
                assert np.array_equal(s[k], ref_state[m][k])
        # eager work between replays
        B.anneal(betas[:3], 1, O.NEAREST_INT, use_graph=False)
    B.close()


def test_batch_matches_oracle_on_small_runs():
    from paper_2401_07965_amd import pa
    betas = schedule(1.0, 6)
    cfgs = configs()[:3]
    B = pa.PABatch(cfgs, max_points=len(betas))
    B.anneal(betas, 2, O.NEAREST_INT, use_graph=True)
    rec = B.records()
    for m, c in enumerate(cfgs):
        o = O.OracleRun(c["dim"], c["L"], c["R"], seed=c["seed"], run_id=c["run_id"],
                        J=c["couplings"])
        for i, b in enumerate(betas[1:], 1):
            assert rel_ok(rec[m, i]["lnQ"], o.reweight(b))
            assert rec[m, i]["R"] == o.resample(O.NEAREST_INT)
            o.sweep(2)
        compare_state(_Exported(B, m), o, f"batch run {m}")
    B.close()


class _Exported:
    def __init__(self, B, m):
        self.B, self.m = B, m

    def export(self):
        return self.B.export_run(self.m)


def test_frozen_run_does_not_disturb_the_others():
    from paper_2401_07965_amd import pa
    betas = [0.0, 0.5, 1.5, 3.0, 4.0]
    cfgs = [dict(dim=2, L=8, R=200, seed=1, run_id=0, couplings=None),
            dict(dim=2, L=4, R=64, seed=5, run_id=0, couplings=None, capacity=64),
            dict(dim=3, L=4, R=300, seed=2, run_id=3, couplings=ea_couplings(3, 4, 1))]
    B = pa.PABatch(cfgs, max_points=len(betas))
    B.anneal(betas, 2, O.POISSON, use_graph=True)
    rec = B.records()
    assert rec[1, -1]["status"] & 16, "the tight-capacity run should freeze"
    for m in (0, 2):
        rows, st = single_records(cfgs[m], betas, 2, O.POISSON)
        assert [r[1] for r in rows] == rec[m]["lnZ"].tolist()
        assert np.array_equal(B.export_run(m)["spins"], st["spins"])
    B.close()


@pytest.mark.parametrize("scheme", [O.NEAREST_INT, O.POISSON, O.SYSTEMATIC, O.MULTINOMIAL])
def test_tile_sizes_follow_each_run_not_the_batch(scheme):
    """The resampling passes tile a run by its own capacity (1024 slots per
    tile below 2^18, 4096 from 2^18 on), so a small run batched with a large
    one, and a large run with capacity just past the switch, give exactly the
    bits of their single runs (copy numbers, sampling variance, state)."""
    from paper_2401_07965_amd import pa
    betas = schedule(1.0, 5)
    cfgs = [dict(dim=2, L=4, R=300, seed=2, run_id=0, couplings=None),
            dict(dim=2, L=4, R=(1 << 18) - 4096, seed=2, run_id=1, couplings=None, capacity=1 << 18),
            dict(dim=2, L=4, R=(1 << 18) - 8192, seed=2, run_id=2, couplings=None, capacity=(1 << 18) - 64)]
    B = pa.PABatch(cfgs, max_points=len(betas))
    B.anneal(betas, 2, scheme, use_graph=False)
    rec = B.records()
    for m, cfg in enumerate(cfgs):
        g = pa.PARun(cfg["dim"], cfg["L"], cfg["R"], seed=cfg["seed"], run_id=cfg["run_id"],
                     capacity=cfg.get("capacity", 0))
        for i, b in enumerate(betas[1:], 1):
            assert rec[m, i]["lnQ"] == g.reweight(b), (m, i)
            assert rec[m, i]["R"] == g.resample(scheme), (m, i)
            g.sweep(2)
            ob = g.observables()
            assert rec[m, i]["sv"] == ob["sv"] and rec[m, i]["lnZ"] == g.free_energy(), (m, i)
        st = g.export()
        bs = B.export_run(m)
        for k in ("spins", "energy", "label"):
            assert np.array_equal(bs[k], st[k]), (m, k)
        g.close()
    B.close()


def test_3d_L16_walks_at_every_size_match_the_oracle():
    """3D L = 16 takes the fixed-axis walk with wave-uniform z offsets at 256,
    512 and 768 lanes (one, two or three z planes of a colour per pass) and
    the general walk at the other sizes; every size gives the oracle's bits."""
    from paper_2401_07965_amd import pa
    betas = [0.0, 0.2, 0.6, 2.6]
    J = ea_couplings(3, 16, 4)
    cfg = dict(dim=3, L=16, R=130, seed=4, run_id=2, couplings=J)
    o = O.OracleRun(3, 16, 130, seed=4, run_id=2, J=J)
    for b in betas[1:]:
        o.reweight(b)
        o.resample(O.SYSTEMATIC)
        o.sweep(2)
    B = pa.PABatch([cfg], max_points=len(betas))
    for t in (256, 512, 768, 192, 640):
        print(f"[batch] 3D L=16 at {t} lanes", flush=True)
        B.set_threads(0, t)
        B.anneal(betas, 2, O.SYSTEMATIC, use_graph=False)
        compare_state(_Exported(B, 0), o, f"3D L=16, {t} lanes")
    B.close()


def test_small_lattices_at_several_walk_sizes_match_the_oracle():
    """Small 2D and 3D glasses at workgroup sizes that give a lane one site of
    a colour (with idle lanes or none) or several, by the fixed-axis walk or
    the general one: every size gives the oracle's bits."""
    from paper_2401_07965_amd import pa
    betas = [0.0, 0.3, 0.9, 2.6]
    cases = [(3, 10, (512, 576, 64, 256)), (3, 8, (256, 128, 320)), (3, 6, (128, 64)),
             (2, 8, (64, 128)), (2, 12, (128, 64)), (2, 16, (128, 64, 192))]
    for d, L, sizes in cases:
        J = ea_couplings(d, L, 5)
        cfg = dict(dim=d, L=L, R=130, seed=6, run_id=1, couplings=J)
        o = O.OracleRun(d, L, 130, seed=6, run_id=1, J=J)
        for b in betas[1:]:
            o.reweight(b)
            o.resample(O.SYSTEMATIC)
            o.sweep(2)
        B = pa.PABatch([cfg], max_points=len(betas))
        for t in sizes:
            print(f"[batch] {d}D L={L} at {t} lanes", flush=True)
            B.set_threads(0, t)
            B.anneal(betas, 2, O.SYSTEMATIC, use_graph=False)
            compare_state(_Exported(B, 0), o, f"{d}D L={L}, {t} lanes")
        B.close()


def test_anneal_without_sweeps_then_export_matches_the_oracle():
    """theta = 0: every step's resampling leaves its spins to be gathered, by
    the next resampling or by the export, eagerly and from a replayed graph."""
    from paper_2401_07965_amd import pa
    betas = [0.0, 0.2, 0.5, 0.9, 1.4]
    J = ea_couplings(3, 6, 8)
    cfgs = [dict(dim=3, L=6, R=300, seed=3, run_id=0, couplings=J), dict(dim=2, L=8, R=200, seed=3, run_id=1)]
    refs = []
    for c in cfgs:
        o = O.OracleRun(c["dim"], c["L"], c["R"], seed=3, run_id=c["run_id"], J=c.get("couplings"))
        for b in betas[1:]:
            o.reweight(b)
            o.resample(O.SYSTEMATIC)
        refs.append(o)
    B = pa.PABatch(cfgs, max_points=len(betas))
    for graph in (False, True, True):
        print(f"[batch] theta = 0, graph={graph}", flush=True)
        B.anneal(betas, 0, O.SYSTEMATIC, use_graph=graph)
        for m, o in enumerate(refs):
            compare_state(_Exported(B, m), o, f"run {m}, theta = 0, graph={graph}")
    B.close()


def test_weighted_combination_matches_oracle():
    from paper_2401_07965_amd import pa
    betas = schedule(1.0, 8)
    J = ea_couplings(2, 8, 9)
    cfgs = [dict(dim=2, L=8, R=int(r), seed=7, run_id=k, couplings=J)
            for k, r in enumerate([300, 500, 800, 1000, 200, 640])]
    B = pa.PABatch(cfgs, max_points=len(betas))
    B.anneal(betas, 3, O.NEAREST_INT, use_graph=True)
    rec = B.records()
    groups = [0, 0, 0, 1, 1, -1]
    for point in (3, 7):
        out = B.combine(groups, 2, point)
        for g in (0, 1):
            rs = [dict(R=int(rec[m, point]["R"]), lnZ=rec[m, point]["lnZ"],
                       beta=rec[m, point]["beta"], e=rec[m, point]["e"], e2=rec[m, point]["e2"],
                       abs_m=rec[m, point]["abs_m"], m2=rec[m, point]["m2"])
                  for m in range(len(cfgs)) if groups[m] == g]
            ref = OC.combine(rs, 64)
            assert out[g]["runs"] == ref["runs"]
            for k in ("lnZ", "e", "e2", "abs_m", "m2", "c", "chi", "n_eff", "c_naive", "chi_naive",
                      "e_plain", "c_plain", "chi_plain"):
                assert rel_ok(out[g][k], ref[k], 1e-12), (point, g, k, out[g][k], ref[k])
    B.close()


def test_tune_at_a_temperature_and_pinned_sizes_change_nothing():
    """The autotuner times every usable workgroup size at the thresholds of a
    given beta and reports the times; any size set by hand gives the same bits."""
    from paper_2401_07965_amd import pa
    betas = schedule(2.0, 9)
    cfgs = configs(seed=6)
    B = pa.PABatch(cfgs, max_points=len(betas))
    B.anneal(betas, 3, O.SYSTEMATIC, use_graph=False)
    ref = B.records().copy()
    chosen, times = B.tune(3, 1.2, times=True)
    for g, t in enumerate(chosen):
        assert t in times[g] and times[g][t] == min(times[g].values()) and times[g][t] > 0
    for g in range(len(chosen)):
        for t in sorted(times[g])[::3]:
            B.set_threads(g, t)
            B.anneal(betas, 3, O.SYSTEMATIC, use_graph=False)
            assert np.array_equal(B.records(), ref), (g, t)
    with pytest.raises(pa.PAError):
        B.set_threads(0, 100)  # not a multiple of 64
    with pytest.raises(pa.PAError):
        B.set_threads(99, 64)  # no such group
    B.close()
