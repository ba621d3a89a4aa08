#!/usr/bin/env python3
"""Throughput of the population-annealing hot path on one MI355X.

Workload (the 2D resampling-scheme study): 2D Ising ferromagnet, L = 64
periodic, target population R = 10^5, theta = 10 checkerboard Metropolis
sweeps per temperature, beta_i = 0.6 i / 200 (201 points), run once with each
of the four resampling schemes (multinomial, Poisson, nearest integer,
systematic; run_id = scheme index, seed 1).  Synthetic lattices, seeded.

One step = one temperature step of all four runs: reweight (Q of Eq. (1)),
resample (copy numbers, prefix sums, gather), theta sweeps, observables.
The runs are independent and each has its own stream, so their kernels
overlap.  ``value`` = spin-flip attempts (theta N R_i summed over the runs)
per ns of wall time over the timed steps, inputs resident in HBM throughout.

Prints one JSON line.  Only one GPU is used; --gpus above 1 is refused.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

D, L, R, THETA, BETA_F, POINTS, SEED = 2, 64, 100000, 10, 0.6, 201, 1
SCHEMES = (("multinomial", 0), ("poisson", 1), ("nearest", 2), ("systematic", 3))

# Roofline of the sweep kernel (integer VALU bound).
# peak = 256 CUs x 64 int32 lanes/clock x 2.4 GHz.  The achieved rate counts
# the fewest 32-bit lane operations known to do the 2D ferromagnet sweep's
# work on gfx950 (three-input bitwise ops), per 64-bit word as two halves:
# each Philox4x32-10 call is 10 rounds of two 32x32->64 multiplies and two
# three-input xors (40); consuming its two bit planes for a 64-replica word is
# 2 planes x 2 halves x (threshold select 1 + accept 1 + undecided 1) plus
# merging the pair's acceptances (2) = 14; a word-site update is the two pair
# sums and two carries of the bonds from the neighbour words (4 x 2), the
# classes u >= 2 and u = 1 and their shared carry (3 x 2) and the flip (2) = 16.
PEAK_INT_OPS = 256 * 64 * 2.4e9
OPS_PER_PHILOX = 40 + 14   # generate a plane pair and decide 64 replicas on it
OPS_PER_SITE_UPDATE = 16   # 2D, no couplings


COUNTER_PROFILE = os.path.join(ROOT, "profiles", "k_sweep_2d_L64_R1e5_counters.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2401_07965_amd", "csrc", f)
                  for f in ("pa_kernels.hip", "pa_device.h", "pa_internal.h")]


def code_only(text):
    """C/C++ source without comments, whitespace collapsed."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    """SHA-256 of the kernel sources' code (code_only), so that a profile
    stays valid across comment edits."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()


def profiled_counters():
    """HBM traffic and VALU figures of the sweep from the committed counter
    profile, or None when the kernel sources changed since it was taken."""
    import re
    try:
        with open(COUNTER_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = dict(re.findall(r"^- (\w+): (\S+)\s*$", text, re.M))
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return vals


def betas():
    return [i * BETA_F / (POINTS - 1) for i in range(POINTS)]


def make_runs(pa, streams=None):
    """The four runs; each on its own stream when streams are given (the runs are
    independent, so one run's small resampling kernels overlap another's sweep)."""
    streams = streams or [None] * len(SCHEMES)
    return [pa.PARun(D, L, R, seed=SEED, run_id=rid, stream=st) for (_, rid), st in zip(SCHEMES, streams)]


def gpu_bench(steps, warmup):
    """Times `steps` temperature steps of the four runs, each run on its own
    stream.  Every call inside the timed region is deferred (nothing waits for
    the device); the sweep and the reweight + resample of each run are
    bracketed by HIP events on the run's stream.  Launches of different runs
    overlap, so kernel time is the union of those intervals over the four
    streams (the time during which that kernel was running).  Attempts and
    work counters come from the device records."""
    import torch
    from paper_2401_07965_amd import pa
    pa.lib()
    sched = betas()
    streams = [torch.cuda.Stream() for _ in SCHEMES]  # default priority
    state = {"i": 0, "runs": make_runs(pa, streams)}
    keys = ("philox_calls", "site_updates", "spin_attempts")
    done = dict.fromkeys(keys, 0)  # counters of runs closed inside the window
    Rsum = {"start": 0, "end": 0}

    def one_step(acc):
        i = state["i"] + 1
        if i == POINTS:  # anneal finished: start the next anneal (step 1 of the method)
            for g in state["runs"]:
                if acc is not None:
                    c = g.counters()
                    for k in keys:
                        done[k] += c[k]
                    Rsum["end"] += g.observables()["R"]
                g.close()
            state["runs"] = make_runs(pa, streams)
            if acc is not None:
                Rsum["start"] += R * len(SCHEMES)
            i = 1
        state["i"] = i
        for (name, rid), g, stream in zip(SCHEMES, state["runs"], streams):
            if acc is None:
                g.reweight(sched[i], wait=False)
                g.resample(rid, wait=False)
                g.sweep(THETA)
                g.observables(wait=False)
                continue
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record(stream)
            g.reweight(sched[i], wait=False)
            g.resample(rid, wait=False)
            ev[1].record(stream)
            g.sweep(THETA)
            ev[2].record(stream)
            g.observables(wait=False)
            acc.append(ev)

    for _ in range(warmup):
        one_step(None)
    base = [g.counters() for g in state["runs"]]  # synchronises; raises if a run failed
    Rsum["start"] += sum(g.observables()["R"] for g in state["runs"])
    acc = []
    torch.cuda.synchronize()
    ref = torch.cuda.Event(enable_timing=True)
    ref.record(streams[0])
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step(acc)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tot = dict(done)
    for g in state["runs"]:
        c = g.counters()
        for k in keys:
            tot[k] += c[k]
        Rsum["end"] += g.observables()["R"]
    # counters of the runs alive at the window start count from their values then
    for b in base:
        for k in keys:
            tot[k] -= b[k]
    sweep_iv = [(ref.elapsed_time(e[1]), ref.elapsed_time(e[2])) for e in acc]
    resample_iv = [(ref.elapsed_time(e[0]), ref.elapsed_time(e[1])) for e in acc]
    iso = isolated_steps(state, streams, sched, ISO_STEPS)
    for g in state["runs"]:
        g.close()
    attempts = tot["spin_attempts"]
    new_replicas = attempts // (THETA * L ** D)
    # replicas before each resampling: the new ones, shifted by one step
    old_replicas = new_replicas + Rsum["start"] - Rsum["end"]
    return dict(elapsed=elapsed, attempts=attempts, sweep_ms=[b - a for a, b in sweep_iv], iso=iso,
                sweep_union_s=union_length(sweep_iv) / 1e3, calls=tot["philox_calls"],
                updates=tot["site_updates"], resample_s=union_length(resample_iv) / 1e3,
                resample_bytes=resample_bytes(old_replicas, new_replicas))


ISO_STEPS = 6


def isolated_steps(state, streams, sched, nsteps):
    """After the timed region (untimed): `nsteps` more steps with one run at a
    time on the device, HIP events around its reweight + resample and its
    sweep.  Gives the per-launch sweep time and the resampling rate without
    the other runs' kernels alongside.  On every other step a gate kernel
    (the generator probe, a few hundred us) runs first on the stream, so that
    the whole reweight + resample is queued before its first kernel starts:
    the rate of the kernels themselves ("pre-queued"); on the others the host
    issues the launches while the device runs them ("host-paced")."""
    import torch
    from paper_2401_07965_amd import pa
    gate = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
    sweep_ms, attempts = [], 0
    res = {True: [0.0, 0.0], False: [0.0, 0.0]}  # pre-queued?: [ms, bytes]
    i = state["i"]
    for k in range(nsteps):
        i += 1
        if i == POINTS:
            break
        queued = k % 2 == 0
        for (name, rid), g, stream in zip(SCHEMES, state["runs"], streams):
            R_old = g.observables()["R"]
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            if queued:
                pa.philox_probe(gate, 128, stream)
            ev[0].record(stream)
            g.reweight(sched[i], wait=False)
            g.resample(rid, wait=False)
            ev[1].record(stream)
            g.sweep(THETA)
            ev[2].record(stream)
            R_new = g.observables()["R"]  # waits for the stream
            res[queued][0] += ev[0].elapsed_time(ev[1])
            res[queued][1] += resample_bytes(R_old, R_new)
            sweep_ms.append(ev[1].elapsed_time(ev[2]))
            attempts += THETA * L ** D * R_new
    if not sweep_ms:
        return None

    def rate(q):
        return res[q][1] / (res[q][0] * 1e-3) / 1e9 if res[q][0] > 0 else None
    return {"steps": len(sweep_ms) // len(SCHEMES),
            "sweep_attempts_per_ns": attempts / (sum(sweep_ms) * 1e-3) / 1e9,
            "sweep_avg_launch_ms": sum(sweep_ms) / len(sweep_ms),
            "resample_GB_per_s": rate(True),
            "resample_GB_per_s_host_paced": rate(False)}


def philox_rate():
    """Device Philox4x32-10 evaluations per second (the library's probe: three
    independent chains per thread, 2^20 threads), best of three timed launches."""
    import torch
    from paper_2401_07965_amd import pa
    out = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    iters = 64
    pa.philox_probe(out, iters, stream)  # warm-up
    best = None
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pa.philox_probe(out, iters, stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return out.numel() * 3 * iters / (best * 1e-3)


def union_length(intervals):
    """Total length of the union of (start, end) intervals."""
    tot, cur_a, cur_b = 0.0, None, None
    for a, b in sorted(intervals):
        if cur_b is None or a > cur_b:
            if cur_b is not None:
                tot += cur_b - cur_a
            cur_a, cur_b = a, b
        else:
            cur_b = max(cur_b, b)
    if cur_b is not None:
        tot += cur_b - cur_a
    return tot


def resample_bytes(R_old, R_new):
    """Algorithmic HBM bytes of reweighting and resampling: per
    old replica the energy read and the copy number / offset writes and reads;
    per new replica the spins read and written (2 N/8 bytes) plus energy,
    magnetisation and label read and written."""
    N = L ** D
    return R_old * (4 + 4 + 4 + 4 + 4) + R_new * (2 * N / 8 + 3 * 4 * 2 + 4)


def resample_scaling(sizes=(100000, 1000000, 4000000), steps=4):
    """Reweight + resample rate against the population size: one run of the
    2D ferromagnet L = 64 per size, theta = 10 sweeps between steps (beta_i =
    0.6 i/200 from i = 100), nearest-integer and systematic resampling, each
    step queued whole behind a gate kernel; HIP events on the run's stream."""
    import torch
    from paper_2401_07965_amd import pa
    gate = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
    sched = betas()
    out = {}
    for R in sizes:
        row = {}
        for name, rid in (("nearest", 2), ("systematic", 3)):
            stream = torch.cuda.Stream()
            g = pa.PARun(D, L, R, seed=1, run_id=rid, stream=stream)
            i0 = 100
            for i in range(1, i0):  # reach the schedule point untimed (one sweep per step)
                g.reweight(sched[i], wait=False)
                g.resample(rid, wait=False)
                g.sweep(1)
            ms, nbytes = 0.0, 0.0
            for i in range(i0, i0 + steps):
                R_old = g.observables()["R"]
                pa.philox_probe(gate, 128, stream)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                g.reweight(sched[i], wait=False)
                g.resample(rid, wait=False)
                e1.record(stream)
                g.sweep(THETA)
                R_new = g.observables()["R"]
                ms += e0.elapsed_time(e1)
                nbytes += resample_bytes(R_old, R_new)
            g.close()
            row[name] = {"GB_per_s": nbytes / (ms * 1e-3) / 1e9, "us_per_resampling": ms * 1e3 / steps}
        out[str(R)] = row
    return {"workload": "2D Ising FM L=64, one run per size, steps at beta_i = 0.6 i/200 from i = 100, "
                        "theta=10, each reweight + resample queued whole", "by_R": out}


def batched_bench(theta=10, scheme=3, verify_runs=8):
    """Uneven-batch workload: 256 independent +-J runs (16 disorder samples x 16
    runs; per sample d in {2,3}, L in {8,12,16,24}; R log-uniform in [1e3, 1e5]),
    beta_i = 3 i/150, theta = 10, systematic resampling.  Times one whole anneal
    of all runs as one HIP graph, the same eagerly, and the same runs one after
    the other through the single-run calls; the results are bit-identical.
    Then, per disorder sample, one run of the sample's total size (Fig. 7's
    alternative to combining M runs): its wall time and the ln Z difference
    from the weighted combination."""
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa, workloads
    cfgs, groups = workloads.uneven_batch()
    betas = workloads.linear_schedule(3.0, 151)
    B = pa.PABatch(cfgs, max_points=len(betas))
    threads = B.tune(theta)
    attempts = theta * sum(c["L"] ** c["dim"] * c["R"] for c in cfgs) * (len(betas) - 1)
    out = {}
    for mode, graph in (("graph", True), ("eager", False)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.anneal(betas, theta, scheme, use_graph=graph)
        torch.cuda.synchronize()
        out[mode] = time.perf_counter() - t0
    rec = B.records()
    comb = B.combine(groups, max(groups) + 1, len(betas) - 1)
    frozen = int(np.sum(rec[:, -1]["status"] & 16 != 0))
    B.close()
    # one run per disorder sample of the runs' total size (Fig. 7's alternative)
    nsamp = max(groups) + 1
    big_cfgs = []
    for s in range(nsamp):
        mine = [c for c, gs in zip(cfgs, groups) if gs == s]
        big_cfgs.append(dict(dim=mine[0]["dim"], L=mine[0]["L"], R=sum(c["R"] for c in mine), seed=2, run_id=s,
                             couplings=mine[0]["couplings"]))
    G = pa.PABatch(big_cfgs, max_points=len(betas))
    G.tune(theta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.anneal(betas, theta, scheme, use_graph=True)
    torch.cuda.synchronize()
    big_s = time.perf_counter() - t0
    grec = G.records()
    G.close()
    dlnz = [abs(comb[s]["lnZ"] - float(grec[s, -1]["lnZ"])) / (big_cfgs[s]["L"] ** big_cfgs[s]["dim"])
            for s in range(nsamp)]
    # the same runs one by one (plain per-run PA through the single-run calls)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    identical = True
    for m, c in enumerate(cfgs):
        g = pa.PARun(c["dim"], c["L"], c["R"], seed=c["seed"], run_id=c["run_id"],
                     couplings=c["couplings"])
        for b in betas[1:]:
            g.reweight(b)
            g.resample(scheme)
            g.sweep(theta)
            g.observables()
        if m < verify_runs:
            identical &= g.free_energy() == rec[m, -1]["lnZ"]
        g.close()
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    return {
        "workload": "256 +-J runs (16 samples x 16), d in {2,3}, L in {8,12,16,24}, "
                    "R log-uniform [1e3,1e5], beta 0->3 in 151 points, theta=10, systematic",
        "runs": len(cfgs), "attempts_per_anneal": attempts,
        "graph_s": out["graph"], "eager_s": out["eager"], "sequential_s": seq,
        "attempts_per_ns_graph": attempts / out["graph"] / 1e9,
        "attempts_per_ns_sequential": attempts / seq / 1e9,
        "speedup_graph_vs_sequential": seq / out["graph"],
        "identical_to_sequential": bool(identical), "frozen_runs": frozen,
        "tuned_threads": threads,
        "combined_lnZ_per_spin_sample0": comb[0]["lnZ"] / (cfgs[0]["L"] ** cfgs[0]["dim"]),
        "mean_n_eff": float(np.mean([c["n_eff"] for c in comb])),
        # per sample, one run of the 16 runs' total size, annealed as a batch of 16
        "one_large_run_per_sample_s": big_s,
        "weighted_vs_large_run_lnZ_per_spin": {"mean_abs_diff": float(np.mean(dlnz)),
                                                "max_abs_diff": float(np.max(dlnz))},
    }


def combination_study(L=16, R=100, theta=1, runs=1024, points=21, beta_f=0.44):
    """Weighted combination of M runs (Sec. 4): 1024 seeded 2D ferromagnet runs
    far from equilibrium (R = 100, theta = 1, 21 temperature points to beta
    0.44), one batched anneal; then for M in 1, 4, 16, 64, 256 the runs are
    combined in groups of M and each estimator is averaged over the groups.
    The reference is the weighted combination of all runs (the most accurate
    estimate available here; the tests compare with the exact values)."""
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa, workloads
    betas = workloads.linear_schedule(beta_f, points)
    cfgs = [dict(dim=2, L=L, R=R, seed=11, run_id=k, couplings=None) for k in range(runs)]
    B = pa.PABatch(cfgs, max_points=len(betas))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.anneal(betas, theta, 3, use_graph=True)
    torch.cuda.synchronize()
    anneal_s = time.perf_counter() - t0
    point = len(betas) - 1
    ref = B.combine([0] * runs, 1, point)[0]
    table = {}
    for M in (1, 4, 16, 64, 256):
        out = B.combine([k // M for k in range(runs)], runs // M, point)
        table[M] = {key: float(np.mean([o[key] for o in out]) - ref[ref_key])
                    for key, ref_key in (("e", "e"), ("e_plain", "e"), ("c", "c"), ("c_naive", "c"),
                                         ("c_plain", "c"))}
    B.close()
    return {"workload": f"{runs} runs 2D Ising FM L={L}, R={R}, theta={theta}, beta 0->{beta_f} in "
                        f"{points} points, systematic; groups of M combined",
            "anneal_s": anneal_s, "reference_e": ref["e"], "reference_c": ref["c"],
            "deviation_from_reference": table}


def resampling_study():
    """Resampling diagnostics per scheme (Sec. 3): the sampling variance of
    Eq. (5) along beta_i = i/300 (2D FM L = 64, R = 2 10^4, theta = 5, up to
    beta = 0.6), and the resampling cost d rho_t / d beta over beta 0 -> 0.3
    for temperature steps from 0.0005 to 0.03 (2D FM L = 32, R = 2 10^4,
    theta = 5)."""
    import numpy as np
    from paper_2401_07965_amd import pa
    t0 = time.perf_counter()
    sv = {}
    for name, sc in SCHEMES:
        g = pa.PARun(2, 64, 20000, seed=3, run_id=sc)
        vals = []
        for i in range(1, 181):
            g.reweight(i / 300.0, wait=False)
            g.resample(sc, wait=False)
            g.sweep(5)
            o = g.observables()
            vals.append((i / 300.0, o["sv"]))
        g.close()
        a = np.array(vals)
        near = a[(a[:, 0] > 0.40) & (a[:, 0] < 0.48)]
        sv[name] = {"mean": float(a[:, 1].mean()), "near_beta_c": float(near[:, 1].mean())}
    cost = {}
    for name, sc in SCHEMES:
        cost[name] = {}
        for db in (0.0005, 0.001, 0.002, 0.005, 0.01, 0.03):
            n = int(round(0.3 / db))
            g = pa.PARun(2, 32, 20000, seed=5, run_id=100 + sc)
            for i in range(1, n + 1):
                g.reweight(i * db, wait=False)
                g.resample(sc, wait=False)
                g.sweep(5)
            cost[name][str(db)] = (g.observables()["rho_t"] - 1.0) / 0.3
            g.close()
    return {"sampling_variance": sv, "resampling_cost_drho_dbeta": cost, "wall_s": time.perf_counter() - t0}


def conditional_study(L=32, R=20000, theta=10, points=101, beta_f=0.44, seeds=8):
    """Conditional resampling (Sec. 3): resample only when the effective sample
    size of the importance weights falls below kappa R.  2D FM L = 32,
    R = 2 10^4, theta = 10, 100 steps to beta = 0.44, systematic, 8 seeds per
    kappa: resamplings per anneal, mean and spread of ln Z_hat over the seeds
    (the tests compare with the exact value), final ESS, anneal time."""
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa
    betas = [i * beta_f / (points - 1) for i in range(points)]
    table = {}
    for kappa in (1.0, 0.9, 0.5, 0.2, 0.0):
        lnz, res, ess, ms = [], [], [], []
        for s in range(seeds):
            g = pa.PARun(2, L, R, seed=31, run_id=s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for b in betas[1:]:
                g.reweight(b, wait=False)
                g.resample_conditional(3, kappa, wait=False)
                g.sweep(theta)
            lnz.append(g.free_energy())
            ms.append((time.perf_counter() - t0) * 1e3)
            res.append(g.counters()["resamplings"])
            ess.append(g.observables()["ess"])
            g.close()
        table[str(kappa)] = {"resamplings": float(np.mean(res)), "lnZ_mean": float(np.mean(lnz)),
                             "lnZ_sd": float(np.std(lnz)), "final_ess": float(np.mean(ess)),
                             "anneal_ms": float(np.mean(ms))}
    return {"workload": f"2D Ising FM L={L}, R={R}, theta={theta}, beta 0->{beta_f} in {points} "
                        f"points, systematic, {seeds} seeds per kappa", "by_kappa": table}


def scheme_error_study(L=64, R=20000, theta=5, runs=128):
    """Fig. 3's workload: specific heat per resampling scheme, 2D FM L = 64,
    R = 2 10^4, theta = 5, beta_i = i/300 to 0.6, 128 seeded runs per scheme
    (one batched anneal each).  Reported: the relative spread of c over the
    runs (statistical error of one run) averaged over beta 0.40..0.47, and the
    anneal time.  The tests compare with the exact c."""
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa
    betas = [i / 300 for i in range(181)]
    N = L * L
    out = {}
    for name, sc in SCHEMES:
        cfgs = [dict(dim=2, L=L, R=R, seed=41, run_id=100 * sc + k, couplings=None) for k in range(runs)]
        B = pa.PABatch(cfgs, max_points=len(betas))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.anneal(betas, theta, sc, use_graph=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = B.records()
        B.close()
        rel = []
        for i in range(120, 142):
            r = rec[:, i]
            Rr = r["R"].astype(np.float64)
            m1 = r["sum_E"] / Rr
            c = betas[i] ** 2 * (r["sum_E2"] / Rr - m1 * m1) / N
            rel.append(float(c.std() / c.mean()))
        out[name] = {"relative_sd_c_near_beta_c": float(np.mean(rel)), "anneal_s": dt}
    return {"workload": f"{runs} runs per scheme, 2D Ising FM L={L}, R={R}, theta={theta}, "
                        f"beta_i = i/300 to 0.6", "by_scheme": out}


def cluster_study(L=64, R=100000, beta_c=0.4406868, updates=10):
    """The cluster-update driver (Wolff updates, pa_cluster) beside Metropolis
    sweeps on the bench lattice at beta_c: time per update of all R replicas,
    mean cluster size (spins that flip, from the exported states), and the
    autocorrelation across the population of E and |m| after k updates of
    either kind, from the same annealed starting population."""
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa
    st = torch.cuda.current_stream()

    def annealed():
        g = pa.PARun(D, L, R, seed=5, run_id=0)
        for i in range(1, 21):
            g.reweight(beta_c * i / 20, wait=False)
            g.resample(3, wait=False)
            g.sweep(2)
        return g

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        fn()
        e1.record(st)
        e1.synchronize()
        return e0.elapsed_time(e1)

    out = {"workload": f"2D Ising FM L={L}, R={R}, beta={beta_c} after 20 annealing steps (theta=2), "
                       "one run per driver from the same seed"}
    corr = {}
    for name in ("cluster", "metropolis"):
        g = annealed()
        step = g.cluster if name == "cluster" else g.sweep
        step(1)  # warm
        out[f"ms_per_{name}_update"] = min(timed(lambda: step(5)) for _ in range(3)) / 5
        s0 = g.export()
        E0 = s0["energy"].astype(np.float64)
        m0 = np.abs(s0["magnetization"]).astype(np.float64)
        ce, cm = [], []
        for k in range(1, updates + 1):
            step(1)
            sk = g.export()
            if k == 1:
                flips = np.unpackbits((s0["spins"] ^ sk["spins"]).view(np.uint8)).sum()
                out[f"{name}_mean_flipped_fraction"] = float(flips) / (R * L ** D)
            ce.append(float(np.corrcoef(E0, sk["energy"].astype(np.float64))[0, 1]))
            cm.append(float(np.corrcoef(m0, np.abs(sk["magnetization"]).astype(np.float64))[0, 1]))
        corr[name] = {"energy": ce, "abs_m": cm}
        g.close()
    out["autocorrelation_after_k_updates"] = corr
    out["cluster_flipped_spins_per_ns"] = (out["cluster_mean_flipped_fraction"] * R * L ** D
                                           / (out["ms_per_cluster_update"] * 1e6))
    return out


def rmsd_study(L=64, R=20000, theta=2, runs=500):
    """Fig. 8's workload: 500 seeded runs of the 2D FM L = 64, R = 2 10^4,
    theta = 2, beta_i = i/300 to 0.6, systematic, one batched anneal; groups of
    M runs combined plainly and by weight.  The reference here is the weighted
    combination of all runs (the tests use the exact values); reported: RMSD of
    u and c at beta = 0.44 and 0.46 for M = 1, 10, 50."""
    import math
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa
    betas = [i / 300 for i in range(181)]
    cfgs = [dict(dim=2, L=L, R=R, seed=43, run_id=k, couplings=None) for k in range(runs)]
    B = pa.PABatch(cfgs, max_points=len(betas))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.anneal(betas, theta, 3, use_graph=True)
    torch.cuda.synchronize()
    anneal_s = time.perf_counter() - t0
    table = {}
    for i in (132, 138):
        ref = B.combine([0] * runs, 1, i)[0]
        row = {}
        for M in (1, 10, 50):
            out = B.combine([k // M for k in range(runs)], runs // M, i)

            def rm(key, rkey):
                return math.sqrt(float(np.mean([(o[key] - ref[rkey]) ** 2 for o in out])))
            row[M] = {"u_plain": rm("e_plain", "e"), "u_weighted": rm("e", "e"),
                      "c_plain": rm("c_plain", "c"), "c_weighted": rm("c", "c")}
        table[f"beta={betas[i]:.3f}"] = row
    B.close()
    return {"workload": f"{runs} runs 2D Ising FM L={L}, R={R}, theta={theta}, beta_i = i/300, "
                        "systematic; groups of M", "anneal_s": anneal_s, "rmsd_vs_all_runs_weighted": table}


def learned_bench(theta=10, scheme=3, astar=0.7, dmax=0.2, beta_f=3.0):
    """Learned-schedule workload: 3D +-J glass L = 16.  The model is trained on
    the GPU from rule-driven anneals of 8 other disorder samples at R = 10^4;
    then the evaluation sample is annealed at R = 10^6 (and 10^4) with the
    rule alone and with the learned step (exact overlap check + rule fallback)."""
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa, workloads
    from paper_2401_07965_amd.schedule import anneal_adaptive, standardisation
    d, L = 3, 16
    Xs, ys = [], []
    t0 = time.perf_counter()
    for s in range(2, 10):
        run = pa.PARun(d, L, 10000, seed=1, run_id=0, couplings=workloads.pm_j_couplings(d, L, s))
        out = anneal_adaptive(run, beta_f, astar, dmax, theta, scheme, record=True)
        Xs.append(out["X"])
        ys.append(out["y"])
        run.close()
    X, y = np.concatenate(Xs), np.concatenate(ys)
    t_data = time.perf_counter() - t0
    xm, xs, ym, ysd = standardisation(X, y)
    mlp = pa.PAMlp(workloads.mlp_initial_parameters(0), xm, xs, ym, ysd, max_samples=len(y))
    mlp.set_data(X, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = mlp.train(2000, 3e-3)
    t_train = time.perf_counter() - t0
    J = workloads.pm_j_couplings(d, L, 1)
    res = {"training_steps": int(len(y)), "train_loss": loss, "data_s": t_data, "train_s": t_train}
    for R in (1000000, 10000):
        for name, model in (("rule", None), ("learned", mlp)):
            run = pa.PARun(d, L, R, seed=1, run_id=0, couplings=J)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = anneal_adaptive(run, beta_f, astar, dmax, theta, scheme, mlp=model)
            torch.cuda.synchronize()
            res[f"R{R}_{name}"] = dict(wall_s=time.perf_counter() - t0, steps=out["steps"],
                                       schedule_s=out["schedule_s"], fallbacks=out["fallbacks"],
                                       lnZ_per_spin=out["lnZ"] / L ** d)
            run.close()
        r, l = res[f"R{R}_rule"], res[f"R{R}_learned"]
        res[f"R{R}_wall_speedup"] = r["wall_s"] / l["wall_s"]
        res[f"R{R}_schedule_speedup"] = r["schedule_s"] / l["schedule_s"]
    mlp.close()
    res["workload"] = ("3D +-J L=16, beta 0->3, alpha*=0.7, dbeta_max=0.2, theta=10, systematic; "
                       "trained on 8 other samples at R=1e4")
    return res


def profile_run():
    """Workload for counter passes: the sweep, resample and observables kernels
    of 3 temperature steps of one run, then torch's copy of 256 MiB (reads and
    writes 2^28 bytes each) as the reference of known traffic."""
    import torch
    from paper_2401_07965_amd import pa
    g = pa.PARun(D, L, R, seed=SEED, run_id=3)
    sched = betas()
    for i in range(1, 4):
        g.reweight(sched[i])
        g.resample(3)
        g.sweep(THETA)
        g.observables()
    torch.cuda.synchronize()
    src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    g.close()
    print("profile run done", flush=True)


def cpu_baseline(budget_s=15.0):
    """The oracle as it stands, on a sample of the same workload: a population
    of R_s = 2048 replicas (same lattice, theta, schedule), whole steps."""
    from oracle import oracle as O
    Rs = 2048
    sched = betas()
    run = O.OracleRun(D, L, Rs, seed=SEED, run_id=3)
    t0 = time.perf_counter()
    attempts = 0
    i = 0
    while True:
        i += 1
        run.reweight(sched[i])
        Rn = run.resample(O.SYSTEMATIC)
        run.sweep(THETA)
        run.observables()
        attempts += THETA * (L ** D) * Rn
        if time.perf_counter() - t0 > budget_s or i == POINTS - 1:
            break
    el = time.perf_counter() - t0
    return {"value": attempts / el / 1e9, "unit": "attempts/ns", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"{i} temperature steps of one systematic-resampling run with R = {Rs} "
                      f"replicas of the same L = 64 lattice, theta = {THETA}, beta_i = 0.6 i/200 "
                      f"({el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=190)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the batched and learned-schedule measurements")
    ap.add_argument("--profile", action="store_true",
                    help="short run for hardware counters: 3 steps of one run of the workload, "
                         "then a 256 MiB device-to-device copy of known size")
    a = ap.parse_args()
    if a.profile:
        profile_run()
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(this library runs one GPU; sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    r = gpu_bench(a.steps, a.warmup)
    rate = philox_rate()
    value = r["attempts"] / r["elapsed"] / 1e9
    # the sweep kernel's time: union of its launches on the four streams
    sweep_s = r["sweep_union_s"]
    avg_launch = sweep_s / len(r["sweep_ms"])
    ops = OPS_PER_PHILOX * r["calls"] + OPS_PER_SITE_UPDATE * r["updates"]
    achieved = ops / sweep_s if r["calls"] else None
    out = {
        "metric": "spin-flip attempts/ns (whole PA temperature step)",
        "value": value,
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r["elapsed"] / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "2D Ising ferromagnet L=64 periodic, R=100000, theta=10, "
                        "beta_i=0.6 i/200 (201 points), four runs: multinomial, Poisson, "
                        "nearest-integer, systematic resampling",
            "dim": D, "L": L, "R": R, "theta": THETA, "runs_per_step": len(SCHEMES),
        },
        "sweep_attempts_per_ns": r["attempts"] / sweep_s / 1e9,
        # reweight + resample rate with one run on the device at a time (the
        # concurrent runs' sweeps stretch its intervals inside the timed region)
        "resample_GB_per_s": r["iso"]["resample_GB_per_s"] if r["iso"] else None,
        "isolated": r["iso"],
        "philox_calls_per_attempt": (r["calls"] / (64.0 * r["updates"])) if r["updates"] else None,
        "philox_calls_per_ns": rate / 1e9,
        # the sweep's rate if generating its random bits were all it did
        "philox_bound_attempts_per_ns": (rate / (r["calls"] / (64.0 * r["updates"])) / 1e9)
                                        if r["updates"] else None,
        "roofline": {
            "kernel": "k_sweep<2>",
            "bound": "alu",
            "achieved": achieved / 1e12 if achieved else None,
            "peak": PEAK_INT_OPS / 1e12,
            "unit": "Tops/s (int32)",
            "frac": achieved / PEAK_INT_OPS if achieved else None,
            "avg_launch_ms": avg_launch * 1e3,
            "concurrent_streams": len(SCHEMES),
            "launch_span_ms": sum(r["sweep_ms"]) / len(r["sweep_ms"]),
            "traffic": None,
        },
    }
    prof = profiled_counters()
    if prof:
        # HBM bytes per sweep launch (FETCH_SIZE, WRITE_SIZE scaled by a copy of known size)
        out["roofline"]["traffic"] = float(prof["traffic_bytes_per_launch"])
        out["roofline"]["traffic_unit"] = "bytes/launch"
        out["roofline"]["valu_busy"] = float(prof["valu_busy"])
    if not a.no_rows:
        out["resample_scaling"] = resample_scaling()
        out["batched"] = batched_bench()
        out["learned"] = learned_bench()
        out["combination"] = combination_study()
        out["resampling"] = resampling_study()
        out["conditional"] = conditional_study()
        out["scheme_errors"] = scheme_error_study()
        out["rmsd"] = rmsd_study()
        out["cluster"] = cluster_study()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
