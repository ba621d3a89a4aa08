#!/usr/bin/env python3
"""Throughput of the population-annealing hot path on one MI355X.

Headline workload (the largest single-run configuration, the learned-schedule
study's system): 3D +-J Edwards-Anderson spin glass, L = 16 periodic
(N = 4096), couplings -1 with probability 1/2 from seed 1, target population
R = 10^6 replicas (15 625 words of 64), theta = 10 checkerboard Metropolis
sweeps per temperature, beta_i = 3 i / 300 (301 points), systematic
resampling, seed 1, run_id 0.  Synthetic, seeded.

One step = one temperature step of the run: reweight (Q of Eq. (1)),
resample (copy numbers, prefix sums, gather), theta sweeps, observables, all
enqueued without a host wait on the run's stream.  ``value`` = spin-flip
attempts (theta N R_i, from the device's own counters) per ns of wall time
over the timed steps, inputs resident in HBM throughout.

Beside the headline: the sweep kernel's roofline (its rate against the
Philox-generation bound, the binding ceiling, and its HBM rate), the whole
anneal, the other workloads (2D ferromagnet with the four schemes and their
free-energy errors against the exact partition function; two 3D glass
populations with ln Q per step and P(q); the uneven batch; the learned
schedule at equal free-energy error) and the paper's figure studies.

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

# headline workload: 3D +-J glass L = 16, R = 10^6
D, L, R, THETA, BETA_F, POINTS, SEED, COUPLING_SEED = 3, 16, 1000000, 10, 3.0, 301, 1, 1
SCHEME = 3  # systematic
SCHEMES = (("multinomial", 0), ("poisson", 1), ("nearest", 2), ("systematic", 3))

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
PEAK_INT_OPS = 256 * 64 * 2.4e9  # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, int32 lane-ops/s
OPS_PER_PHILOX = 40              # 10 rounds x (2 wide multiplies + 2 three-input xors)

# Op model (a lower-bound instruction price, reported beside the roofline):
# per Philox call, generating its two planes (40) and deciding the 64
# replicas of a word on them: per plane and half-word a class-threshold
# select (2 three-input ops in 3D, 1 in 2D), the acceptance and the
# undecided update (2), then merging the pair's acceptances (2); per
# word-site update the bonds, the energy-change classes and the flip.
OP_MODEL = {
    "3d_pmj": {"per_philox": 40 + 2 * 2 * (2 + 2) + 2, "per_site_update": 6 * 3 + 26 + 2},
    "2d_fm": {"per_philox": 40 + 2 * 2 * (1 + 2) + 2, "per_site_update": 16},
}

PROFILE_DIR = os.path.join(ROOT, "profiles")
COUNTER_PROFILES = {
    "glass3d_L16": os.path.join(PROFILE_DIR, "k_sweep_3d_pmj_L16_R1e6_counters.md"),
    "glass3d_L10": os.path.join(PROFILE_DIR, "k_sweep_3d_pmj_L10_R5e5_counters.md"),
    "fm2d_L64": os.path.join(PROFILE_DIR, "k_sweep_2d_fm_L64_R1e5_counters.md"),
}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2401_07965_amd", "csrc", f)
                  for f in ("pa_kernels.hip", "pa_sweep.h", "pa_sweep3.hip", "pa_device.h", "pa_internal.h")]
KAUFMAN_L64 = os.path.join(ROOT, "tests", "golden", "kaufman_2d_L64.json")


def code_only(text):
    """C/C++ source without comments, whitespace collapsed."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    """SHA-256 of the kernel sources' code (code_only) and of the build's
    code-generation flags, so that a profile stays valid across comment
    edits and no longer once the generated code can differ."""
    import hashlib
    from paper_2401_07965_amd import build as B
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    h.update(repr((B.COMMON, sorted(B.FILE_FLAGS.items()))).encode())
    return h.hexdigest()


def profiled_counters(which):
    """The machine-readable figures of a committed counter profile, or None
    when the kernel sources changed since it was taken."""
    import re
    try:
        with open(COUNTER_PROFILES[which]) as fh:
            text = fh.read()
    except (OSError, KeyError):
        return None
    vals = dict(re.findall(r"^- (\w+): (\S+)\s*$", text, re.M))
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return vals


def schedule(beta_f=BETA_F, points=POINTS):
    return [i * beta_f / (points - 1) for i in range(points)]


def headline_couplings():
    from paper_2401_07965_amd import workloads
    return workloads.pm_j_couplings(D, L, COUPLING_SEED)


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


def resample_bytes(N, R_old, R_new):
    """Algorithmic HBM bytes of reweighting and resampling (a fixed model of
    the work, kept across implementations): per old replica 20 B (its energy
    read, a copy number or weight written and read, the ancestor map
    written); per new replica its spins read and written (2 N/8 B) plus
    energy, magnetisation and label read and written and the ancestor read
    (28 B)."""
    return R_old * (4 + 4 + 4 + 4 + 4) + R_new * (2 * N / 8 + 3 * 4 * 2 + 4)


def sweep_bytes(N, words):
    """Algorithmic HBM bytes of one sweep launch over `words` 64-replica
    columns: each column's spins read once and written once (the theta sweeps
    run in LDS), and every replica's energy and magnetisation written."""
    return words * (2 * N * 8 + 64 * 8)


class Step:
    """Deferred temperature steps of one run on its stream, with HIP events
    around its reweight + resample and its sweep (the stream the kernels run
    on: torch.cuda.Event records on the stream it is given)."""

    def __init__(self, make_run, sched, stream):
        self.make_run, self.sched, self.stream = make_run, sched, stream
        self.run = make_run()
        self.i = 0
        self.closed = {"philox_calls": 0, "site_updates": 0, "spin_attempts": 0}
        self.restarts = 0

    def __call__(self, events=None):
        import torch
        i = self.i + 1
        if i == len(self.sched):  # anneal finished: start the next one (step 1 of the method)
            c = self.run.counters()
            for k in self.closed:
                self.closed[k] += c[k]
            self.run.close()
            self.run = self.make_run()
            self.restarts += 1
            i = 1
        self.i = i
        g = self.run
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)] if events is not None else None
        if ev:
            ev[0].record(self.stream)
        g.reweight(self.sched[i], wait=False)
        g.resample(SCHEME, wait=False)
        if ev:
            ev[1].record(self.stream)
        g.sweep(THETA)
        if ev:
            ev[2].record(self.stream)
        g.observables(wait=False)
        if ev:
            events.append((i, ev))

    def totals(self):
        c = self.run.counters()
        return {k: self.closed[k] + c[k] for k in self.closed}


def make_headline_run(stream):
    from paper_2401_07965_amd import pa
    J = headline_couplings()
    return lambda: pa.PARun(D, L, R, seed=SEED, run_id=0, couplings=J, stream=stream)


def headline_bench(steps, warmup):
    """The timed region: `steps` temperature steps of the headline run after
    `warmup` untimed ones, bracketed by device synchronisations.  Sweep and
    resampling kernel times come from HIP events on the run's stream; the
    counts of attempts, Philox evaluations and word-site updates from the
    device records."""
    import torch
    from paper_2401_07965_amd import pa
    pa.lib()
    stream = torch.cuda.Stream()  # default priority
    step = Step(make_headline_run(stream), schedule(), stream)
    for _ in range(warmup):
        step()
    base = step.totals()  # synchronises; raises if the run failed
    ev = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(ev)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tot = step.totals()
    d = {k: tot[k] - base[k] for k in tot}
    sweep_ms = [e[1].elapsed_time(e[2]) for _, e in ev]
    res_ms = [e[0].elapsed_time(e[1]) for _, e in ev]
    words = d["site_updates"] // (THETA * L ** D)  # 64-replica columns swept
    step.run.close()
    return dict(elapsed=elapsed, attempts=d["spin_attempts"], calls=d["philox_calls"],
                updates=d["site_updates"], words=words, sweep_ms=sweep_ms, res_ms=res_ms,
                res_bytes=steps * resample_bytes(L ** D, R, R), restarts=step.restarts,
                beta_range=[schedule()[ev[0][0]], schedule()[ev[-1][0]]] if ev else None)


def anneal_row(rate=None):
    """One whole anneal of the headline workload (300 steps, deferred calls,
    one synchronisation at the end): wall time, attempts per ns, and the sweep
    kernel's rate (HIP events) in windows of beta.  Then the same anneal once
    more with the work counters read at the window boundaries (synchronising
    there): the Philox calls per attempt of each window and, with the
    device's Philox rate, the sweep's fraction of its Philox bound."""
    import torch
    stream = torch.cuda.Stream()
    step = Step(make_headline_run(stream), schedule(), stream)
    ev = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(POINTS - 1):
        step(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot = step.totals()
    lnZ = step.run.free_energy()
    obs = step.run.observables()
    step.run.close()
    att_step = THETA * L ** D * R  # systematic resampling keeps R
    windows, win_ms = {}, {}
    for lo in (0.0, 0.5, 1.0, 1.5, 2.0, 2.5):
        ms = [e[1].elapsed_time(e[2]) for i, e in ev if lo < schedule()[i] <= lo + 0.5 + 1e-12]
        windows[f"({lo:.1f},{lo + 0.5:.1f}]"] = att_step * len(ms) / (sum(ms) * 1e-3) / 1e9
        win_ms[f"({lo:.1f},{lo + 0.5:.1f}]"] = sum(ms)
    by_window = {}
    if rate:
        step2 = Step(make_headline_run(stream), schedule(), stream)
        prev = step2.totals()
        for k, w in enumerate(win_ms):
            for _ in range(50):
                step2()
            cur = step2.totals()
            calls = cur["philox_calls"] - prev["philox_calls"]
            cpa = calls / (64.0 * (cur["site_updates"] - prev["site_updates"]))
            by_window[w] = {"philox_calls_per_attempt": cpa,
                            "philox_bound_attempts_per_ns": rate / cpa / 1e9,
                            "frac": windows[w] * cpa / (rate / 1e9)}
            prev = cur
        step2.run.close()
    sweep_total_ms = sum(e[1].elapsed_time(e[2]) for _, e in ev)
    res_total_ms = sum(e[0].elapsed_time(e[1]) for _, e in ev)
    return {"workload": "the headline workload, one whole anneal beta 0 -> 3 (300 steps)",
            "wall_s": wall, "attempts_per_ns": tot["spin_attempts"] / wall / 1e9,
            "sweep_attempts_per_ns": tot["spin_attempts"] / (sweep_total_ms * 1e-3) / 1e9,
            "sweep_attempts_per_ns_by_beta": windows,
            "philox_bound_by_beta": by_window,
            "sweep_share_of_wall": sweep_total_ms * 1e-3 / wall,
            "resample_GB_per_s": resample_bytes(L ** D, R, R) * (POINTS - 1) / (res_total_ms * 1e-3) / 1e9,
            "philox_calls_per_attempt": tot["philox_calls"] / (64.0 * tot["site_updates"]),
            "lnZ_per_spin_final": lnZ / L ** D, "e_final": obs["e"]}


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


def sweep_roofline(kernel, N, attempts, calls, updates, words, launch_ms, rate, model, profile):
    """Roofline of one sweep kernel.  The sweep is bound by integer VALU work,
    and within it by generating the random bits its decisions need (Philox
    calls counted by the kernel, equal to the oracle's count): the binding
    ceiling is the device's measured Philox rate divided by the calls per
    attempt.  achieved = attempts per launch / mean launch time (HIP events);
    the HBM rate and an instruction-price model are reported beside it."""
    n = len(launch_ms)
    t = sum(launch_ms) * 1e-3
    cpa = calls / (64.0 * updates)
    achieved = attempts / t / 1e9
    peak = rate / cpa / 1e9
    hbm = sweep_bytes(N, words / n) * n / t / 1e9
    ops = OP_MODEL[model]["per_philox"] * calls + OP_MODEL[model]["per_site_update"] * updates
    out = {
        "kernel": kernel, "bound": "alu", "achieved": achieved, "peak": peak, "unit": "attempts/ns",
        "frac": achieved / peak,
        "peak_basis": "measured Philox4x32-10 calls/ns (pa_philox_probe) / Philox calls per attempt "
                      "of these launches",
        "philox_calls_per_ns": rate / 1e9, "philox_calls_per_attempt": cpa,
        "philox_calls_per_ns_chip": PEAK_INT_OPS / OPS_PER_PHILOX / 1e9,
        "attempts_per_launch": attempts / n, "avg_launch_ms": sum(launch_ms) / n, "launches": n,
        "hbm": {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm / HBM_PEAK_GBS,
                "algorithmic_bytes_per_launch": sweep_bytes(N, words / n)},
        "op_model": {"ops_per_philox_call": OP_MODEL[model]["per_philox"],
                     "ops_per_site_update": OP_MODEL[model]["per_site_update"],
                     "achieved_Tops": ops / t / 1e12, "peak_Tops": PEAK_INT_OPS / 1e12,
                     "frac": ops / t / PEAK_INT_OPS},
        "traffic": None,
    }
    if profile:
        out["traffic"] = float(profile["traffic_bytes_per_launch"])
        out["traffic_unit"] = "bytes/launch"
        out["valu_busy"] = float(profile["valu_busy"])
        out["counter_profile"] = os.path.relpath(profile["path"], ROOT)
    return out


def fm2d_L64_row(steps_timed=None):
    """2D Ising ferromagnet L = 64, R = 10^5, theta = 10, beta_i = 0.6 i/200
    (201 points), one run per resampling scheme (run_id = scheme, seed 1),
    each on its own stream: one whole anneal of the four runs (deferred
    calls), its rate and the sweep kernel's (union of its HIP-event intervals
    over the four streams); then per scheme ln Z_hat at beta = 0.6 against
    the exact finite-lattice value (Kaufman), with e, |m|, family entropy and
    rho_t."""
    import torch
    from paper_2401_07965_amd import pa
    d2, L2, R2, bf, pts = 2, 64, 100000, 0.6, 201
    sched = schedule(bf, pts)
    streams = [torch.cuda.Stream() for _ in SCHEMES]
    runs = [pa.PARun(d2, L2, R2, seed=1, run_id=rid, stream=st) for (_, rid), st in zip(SCHEMES, streams)]
    ev = []
    torch.cuda.synchronize()
    ref = torch.cuda.Event(enable_timing=True)
    ref.record(streams[0])
    t0 = time.perf_counter()
    for i in range(1, pts):
        for (name, rid), g, st in zip(SCHEMES, runs, streams):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            g.reweight(sched[i], wait=False)
            g.resample(rid, wait=False)
            e[0].record(st)
            g.sweep(THETA)
            e[1].record(st)
            g.observables(wait=False)
            ev.append(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    with open(KAUFMAN_L64) as f:
        exact = {p["i"]: p for p in json.load(f)["points"]}[pts - 1]
    N2 = L2 * L2
    attempts, calls, updates, by = 0, 0, 0, {}
    for (name, rid), g in zip(SCHEMES, runs):
        c = g.counters()
        attempts += c["spin_attempts"]
        calls += c["philox_calls"]
        updates += c["site_updates"]
        o = g.observables()
        lnz = g.free_energy()
        by[name] = {"lnZ": lnz, "lnZ_exact": exact["lnZ"], "lnZ_error": lnz - exact["lnZ"],
                    "free_energy_error_per_spin": -(lnz - exact["lnZ"]) / (bf * N2),
                    "e": o["e"], "e_exact": exact["e"], "abs_m": o["abs_m"], "S_f": o["S_f"],
                    "rho_t": o["rho_t"], "R": o["R"]}
        g.close()
    union_s = union_length([(ref.elapsed_time(a), ref.elapsed_time(b)) for a, b in ev]) / 1e3
    return {"workload": "2D Ising FM L=64, R=1e5, theta=10, beta_i=0.6 i/200 (201 points), four runs "
                        "(multinomial, Poisson, nearest-integer, systematic), one stream each, one whole anneal",
            "wall_s": wall, "attempts_per_ns": attempts / wall / 1e9,
            "sweep_attempts_per_ns_union": attempts / union_s / 1e9,
            "philox_calls_per_attempt": calls / (64.0 * updates),
            "exact_reference": "Kaufman finite-torus ln Z at beta = 0.6 (tests/golden/kaufman_2d_L64.json)",
            "by_scheme": by}


def glass3d_L10_row():
    """3D +-J glass L = 10, R = 5 10^5 per population, theta = 10,
    beta_i = 3 i/300 (301 points), systematic; populations A and B (run_id 0
    and 1, same couplings from seed 1) annealed together as a batch (one HIP
    graph): wall time, ln Q per step (every 10th step shown, from the step
    records), the energy per spin at beta = 3 and the overlap distribution
    P(q) between A and B at beta = 3; beside it the sweep kernel alone over
    both populations, as the tuner times it at the thresholds of beta = 0.15
    and 1.5."""
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa, workloads
    d3, L3, R3, pts = 3, 10, 500000, 301
    J = workloads.pm_j_couplings(d3, L3, 1)
    sched = schedule(3.0, pts)
    cfgs = [dict(dim=d3, L=L3, R=R3, seed=1, run_id=k, couplings=J) for k in (0, 1)]
    B = pa.PABatch(cfgs, max_points=pts)
    # the sweep alone (both populations in one launch, every workgroup size
    # timed by the tuner) at the thresholds of two temperatures
    N3 = L3 ** d3
    sweep_rate = {}
    for beta in (0.15, 1.5):
        chosen, tab = B.tune(THETA, beta, times=True)
        sweep_rate[str(beta)] = {"threads": chosen[0],
                                 "attempts_per_ns": THETA * N3 * 2 * R3 / (tab[0][chosen[0]] * 1e6)}
    B.anneal(sched, THETA, SCHEME, use_graph=True)  # capture + first launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.anneal(sched, THETA, SCHEME, use_graph=True)  # replay
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rec = B.records()
    h = B.overlap(0, 1)
    B.close()
    q = (2.0 * np.arange(N3 + 1) - N3) / N3
    P = h / h.sum()
    edges = np.linspace(-1, 1, 21)
    hist20 = [float(P[(q >= a) & ((q < b) if b < 1 else (q <= b))].sum()) for a, b in zip(edges[:-1], edges[1:])]
    attempts = THETA * N3 * sum(int(rec[m, i]["R"]) for m in (0, 1) for i in range(1, pts))
    return {"workload": "3D +-J EA L=10 (couplings seed 1), R=5e5 per population, populations A/B "
                        "(run_id 0/1), theta=10, beta_i=3 i/300 (301 points), systematic, one batch "
                        "(graph replay)",
            "wall_s": wall, "attempts_per_ns": attempts / wall / 1e9,
            "sweep_only_by_threshold_beta": sweep_rate,
            "lnQ_every_10th_step": {"A": [float(rec[0, i]["lnQ"]) for i in range(10, pts, 10)],
                                     "B": [float(rec[1, i]["lnQ"]) for i in range(10, pts, 10)]},
            "lnZ_per_spin_final": [float(rec[m, -1]["lnZ"]) / N3 for m in (0, 1)],
            "e_final": [float(rec[m, -1]["e"]) for m in (0, 1)],
            "rho_t_final": [float(rec[m, -1]["rho_t"]) for m in (0, 1)],
            "overlap": {"pairs": int(h.sum()), "mean_abs_q": float((P * np.abs(q)).sum()),
                        "mean_q2": float((P * q * q).sum()),
                        "P_q_20_bins_-1_to_1": hist20}}


def resample_scaling(sizes=(100000, 1000000, 4000000), steps=4):
    """Reweight + resample rate against the population size: one run of the
    2D ferromagnet L = 64 per size, theta = 10 sweeps between steps (beta_i =
    0.6 i/200 from i = 100), nearest-integer and systematic resampling, each
    step queued whole behind a gate kernel; HIP events on the run's stream."""
    import torch
    from paper_2401_07965_amd import pa
    gate = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
    sched = schedule(0.6, 201)
    out = {}
    for Rs in sizes:
        row = {}
        for name, rid in (("nearest", 2), ("systematic", 3)):
            stream = torch.cuda.Stream()
            g = pa.PARun(2, 64, Rs, seed=1, run_id=rid, stream=stream)
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
                nbytes += resample_bytes(64 * 64, R_old, R_new)
            g.close()
            row[name] = {"GB_per_s": nbytes / (ms * 1e-3) / 1e9, "us_per_resampling": ms * 1e3 / steps}
        out[str(Rs)] = row
    return {"workload": "2D Ising FM L=64, one run per size, steps at beta_i = 0.6 i/200 from i = 100, "
                        "theta=10, each reweight + resample queued whole", "by_R": out}


def batched_bench(theta=10, scheme=3, plain_streams=8):
    """Uneven-batch workload: 256 independent +-J runs (16 disorder samples x 16
    runs; per sample d in {2,3}, L in {8,12,16,24}; R log-uniform in [1e3, 1e5]),
    beta_i = 3 i/150, theta = 10, systematic resampling.  One whole anneal of
    all runs: captured as a HIP graph (capture + instantiation + launch), then
    replayed, eagerly, and as plain per-run PA through the single-run calls in
    their fastest form (deferred calls, runs spread over `plain_streams`
    streams so that their kernels overlap).  Every run's final ln Z_hat and
    population are compared with the batch's (identical by construction).
    Then, per disorder sample, one run of the sample's total size (Fig. 7's
    alternative to combining M runs): its wall time and the ln Z difference
    from the weighted combination."""
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa, workloads
    cfgs, groups = workloads.uneven_batch()
    betas = workloads.linear_schedule(3.0, 151)
    B = pa.PABatch(cfgs, max_points=len(betas))
    threads = B.tune(theta, 1.5)
    attempts = theta * sum(c["L"] ** c["dim"] * c["R"] for c in cfgs) * (len(betas) - 1)
    out = {}
    for mode, graph in (("graph_first", True), ("graph_replay", True), ("eager", False)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.anneal(betas, theta, scheme, use_graph=graph)
        torch.cuda.synchronize()
        out[mode] = time.perf_counter() - t0
    rec = B.records()
    comb = B.combine(groups, max(groups) + 1, len(betas) - 1)
    frozen = int(np.sum(rec[:, -1]["status"] & 16 != 0))
    B.close()
    # plain per-run PA: the same runs through the single-run calls, deferred,
    # runs spread round-robin over streams
    streams = [torch.cuda.Stream() for _ in range(plain_streams)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [pa.PARun(c["dim"], c["L"], c["R"], seed=c["seed"], run_id=c["run_id"], couplings=c["couplings"],
                     stream=streams[m % plain_streams]) for m, c in enumerate(cfgs)]
    t_setup = time.perf_counter() - t0
    for b in betas[1:]:
        for g in runs:
            g.reweight(b, wait=False)
            g.resample(scheme, wait=False)
            g.sweep(theta)
            g.observables(wait=False)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    mismatched = 0
    for m, g in enumerate(runs):
        if g.free_energy() != rec[m, -1]["lnZ"] or g.observables()["R"] != rec[m, -1]["R"]:
            mismatched += 1
        g.close()
    # one run per disorder sample of the runs' total size (Fig. 7's alternative)
    nsamp = max(groups) + 1
    big_cfgs = []
    for s in range(nsamp):
        mine = [c for c, gs in zip(cfgs, groups) if gs == s]
        big_cfgs.append(dict(dim=mine[0]["dim"], L=mine[0]["L"], R=sum(c["R"] for c in mine), seed=2, run_id=s,
                             couplings=mine[0]["couplings"]))
    G = pa.PABatch(big_cfgs, max_points=len(betas))
    G.tune(theta, 1.5)
    G.anneal(betas, theta, scheme, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.anneal(betas, theta, scheme, use_graph=True)
    torch.cuda.synchronize()
    big_s = time.perf_counter() - t0
    grec = G.records()
    G.close()
    dlnz = [abs(comb[s]["lnZ"] - float(grec[s, -1]["lnZ"])) / (big_cfgs[s]["L"] ** big_cfgs[s]["dim"])
            for s in range(nsamp)]
    return {
        "workload": "256 +-J runs (16 samples x 16), d in {2,3}, L in {8,12,16,24}, "
                    "R log-uniform [1e3,1e5], beta 0->3 in 151 points, theta=10, systematic",
        "runs": len(cfgs), "attempts_per_anneal": attempts,
        "graph_first_s": out["graph_first"], "graph_replay_s": out["graph_replay"], "eager_s": out["eager"],
        "plain_per_run_s": plain, "plain_per_run_setup_s": t_setup, "plain_streams": plain_streams,
        "attempts_per_ns_graph": attempts / out["graph_replay"] / 1e9,
        "attempts_per_ns_plain_per_run": attempts / plain / 1e9,
        "speedup_graph_vs_plain_per_run": plain / out["graph_replay"],
        "runs_checked_identical": len(cfgs) - mismatched, "runs_mismatched": mismatched,
        "frozen_runs": frozen, "tuned_threads": threads,
        "mean_n_eff": float(np.mean([c["n_eff"] for c in comb])),
        # per sample, one run of the 16 runs' total size, annealed as a batch of 16 (graph replay)
        "one_large_run_per_sample_s": big_s,
        "weighted_vs_large_run_lnZ_per_spin": {"mean_abs_diff": float(np.mean(dlnz)),
                                                "max_abs_diff": float(np.max(dlnz))},
    }


def learned_bench(theta=10, scheme=3, astar=0.7, dmax=0.2, beta_f=3.0, Reval=1000000, Rtrain=10000,
                  runs=16, records=2000, bracket=1.25, refine=6):
    """Learned-schedule workload: 3D +-J glass L = 16, beta 0 -> 3, theta = 10,
    systematic.  Training data: (features, ln dbeta) records of rule-driven
    anneals at R = 10^4 of other disorder samples (coupling seeds 2, 3, ...)
    until `records` records exist; the model is trained on the GPU.
    Evaluation on the sample of coupling seed 1 at R = 10^6: `runs` anneals
    (run_id 0..runs-1) with the overlap rule alone and as many with the
    learned step (the model's proposal refined in a bracket by a few exact
    overlap evaluations, the rule as fallback), both driven by deferred calls
    (only the step choice waits for the device).  Reported per schedule: mean
    and spread of the wall time, steps, fallbacks, the spread of ln Z_hat at
    beta = 3 over the runs and its mean, and the RMSD against the reference,
    the free-energy-weighted combination (Eq. (10), equal R) of all
    2 x `runs` anneals, with standard errors."""
    import numpy as np
    import torch
    from paper_2401_07965_amd import pa, workloads
    from paper_2401_07965_amd.schedule import anneal_adaptive, standardisation
    d, Ls = 3, 16
    Xs, ys = [], []
    t0 = time.perf_counter()
    s = 2
    while sum(len(y) for y in ys) < records:
        run = pa.PARun(d, Ls, Rtrain, seed=1, run_id=0, couplings=workloads.pm_j_couplings(d, Ls, s))
        o = anneal_adaptive(run, beta_f, astar, dmax, theta, scheme, record=True)
        Xs.append(o["X"])
        ys.append(o["y"])
        run.close()
        s += 1
    X, y = np.concatenate(Xs)[:records], np.concatenate(ys)[:records]
    t_data = time.perf_counter() - t0
    xm, xs, ym, ysd = standardisation(X, y)
    mlp = pa.PAMlp(workloads.mlp_initial_parameters(0), xm, xs, ym, ysd, max_samples=len(y))
    mlp.set_data(X, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = mlp.train(2000, 3e-3)
    t_train = time.perf_counter() - t0
    J = workloads.pm_j_couplings(d, Ls, 1)
    res = {"training_records": int(len(y)), "training_samples": s - 2, "train_loss": loss,
           "data_s": t_data, "train_s": t_train}
    per = {}
    for name, model in (("rule", None), ("learned", mlp)):
        wall, steps, sched_s, fb, lnz = [], [], [], [], []
        for k in range(runs):
            run = pa.PARun(d, Ls, Reval, seed=1, run_id=k, couplings=J)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = anneal_adaptive(run, beta_f, astar, dmax, theta, scheme, mlp=model, bracket=bracket,
                                refine=refine, deferred=True, sync=torch.cuda.synchronize)
            torch.cuda.synchronize()
            wall.append(time.perf_counter() - t0)
            steps.append(o["steps"])
            sched_s.append(o["schedule_s"])
            fb.append(o["fallbacks"])
            lnz.append(o["lnZ"])
            run.close()
        per[name] = dict(wall=np.array(wall), steps=np.array(steps), sched=np.array(sched_s),
                         fb=np.array(fb), lnz=np.array(lnz))
    mlp.close()
    allz = np.concatenate([per[n]["lnz"] for n in per])
    ref = float(allz.max() + np.log(np.exp(allz - allz.max()).sum()) - np.log(len(allz)))
    for name, p in per.items():
        dev2 = (p["lnz"] - ref) ** 2
        rmsd = float(np.sqrt(dev2.mean()))
        # standard error of the RMSD from that of the mean squared deviation
        se = float(dev2.std(ddof=1) / np.sqrt(len(dev2)) / (2 * rmsd)) if rmsd > 0 else 0.0
        sd = float(p["lnz"].std(ddof=1))
        res[name] = {"wall_s_mean": float(p["wall"].mean()), "wall_s_sd": float(p["wall"].std(ddof=1)),
                     "steps_mean": float(p["steps"].mean()), "schedule_s_mean": float(p["sched"].mean()),
                     "fallbacks_mean": float(p["fb"].mean()),
                     "lnZ_mean": float(p["lnz"].mean()), "lnZ_mean_se": sd / math.sqrt(len(p["lnz"])),
                     "lnZ_sd": sd, "lnZ_sd_se": sd / math.sqrt(2 * (len(p["lnz"]) - 1)),
                     "rmsd_lnZ": rmsd, "rmsd_lnZ_se": se,
                     "mean_lnZ_minus_reference": float((p["lnz"] - ref).mean())}
    r, l = res["rule"], res["learned"]
    res["wall_speedup"] = r["wall_s_mean"] / l["wall_s_mean"]
    res["wall_speedup_se"] = res["wall_speedup"] * math.hypot(
        r["wall_s_sd"] / math.sqrt(runs) / r["wall_s_mean"], l["wall_s_sd"] / math.sqrt(runs) / l["wall_s_mean"])
    res["rmsd_ratio_learned_over_rule"] = l["rmsd_lnZ"] / r["rmsd_lnZ"] if r["rmsd_lnZ"] > 0 else None
    res["lnZ_sd_ratio_learned_over_rule"] = l["lnZ_sd"] / r["lnZ_sd"] if r["lnZ_sd"] > 0 else None
    res["lnZ_mean_difference"] = l["lnZ_mean"] - r["lnZ_mean"]
    res["lnZ_mean_difference_se"] = math.hypot(l["lnZ_mean_se"], r["lnZ_mean_se"])
    res["learned_step"] = f"proposal refined in a bracket of {bracket} by {refine} halvings, rule as fallback"
    res["reference"] = f"weighted combination (Eq. (10), equal R) of all {2 * runs} anneals' ln Z_hat at beta = 3"
    res["workload"] = (f"3D +-J L=16 (couplings seed 1), R={Reval}, beta 0->3, alpha*={astar}, dbeta_max={dmax}, "
                       f"theta={theta}, systematic; {runs} run_ids per schedule; trained on {len(y)} records of "
                       f"rule-driven anneals at R={Rtrain} of other samples")
    return res


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
        g = pa.PARun(2, L, R, seed=5, run_id=0)
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
                out[f"{name}_mean_flipped_fraction"] = float(flips) / (R * L ** 2)
            ce.append(float(np.corrcoef(E0, sk["energy"].astype(np.float64))[0, 1]))
            cm.append(float(np.corrcoef(m0, np.abs(sk["magnetization"]).astype(np.float64))[0, 1]))
        corr[name] = {"energy": ce, "abs_m": cm}
        g.close()
    out["autocorrelation_after_k_updates"] = corr
    out["cluster_flipped_spins_per_ns"] = (out["cluster_mean_flipped_fraction"] * R * L ** 2
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


def profile_run(which, steps, warmup):
    """Workload for counter passes: `warmup + steps` temperature steps of one
    run of the named workload (deferred calls; the sweep launches of the last
    `steps` are the timed window of the headline), then torch's copy of
    256 MiB (reads and writes 2^28 bytes each) as the reference of known
    traffic."""
    import torch
    from paper_2401_07965_amd import pa, workloads
    if which == "glass3d_L16":
        J, d, Ls, Rs, sched, sc = headline_couplings(), D, L, R, schedule(), SCHEME
    elif which == "glass3d_L10":
        J, d, Ls, Rs, sched, sc = workloads.pm_j_couplings(3, 10, 1), 3, 10, 500000, schedule(3.0, 301), SCHEME
    else:
        J, d, Ls, Rs, sched, sc = None, 2, 64, 100000, schedule(0.6, 201), 3
    g = pa.PARun(d, Ls, Rs, seed=SEED, run_id=0, couplings=J)
    for i in range(1, warmup + steps + 1):
        g.reweight(sched[i], wait=False)
        g.resample(sc, wait=False)
        g.sweep(THETA)
        g.observables(wait=False)
    torch.cuda.synchronize()
    src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    g.close()
    print(f"profile run done: {which}, steps 1..{warmup + steps}", flush=True)


def cpu_baseline(budget_s=12.0, budget_1core_s=6.0):
    """The oracle as it stands, on a sample of the headline workload: a
    population of R_s = 2048 replicas of the same lattice and couplings,
    theta = 10, beta_i = 3 i/300, whole steps (reweight, systematic
    resampling, sweeps, observables) until the time budget is spent; on all
    host threads, then on one."""
    from oracle import oracle as O
    Rs = 2048
    sched = schedule()
    J = headline_couplings()

    def timed(budget):
        run = O.OracleRun(D, L, Rs, seed=SEED, run_id=0, J=J)
        t0 = time.perf_counter()
        attempts, i = 0, 0
        while True:
            i += 1
            run.reweight(sched[i])
            Rn = run.resample(O.SYSTEMATIC)
            run.sweep(THETA)
            run.observables()
            attempts += THETA * (L ** D) * Rn
            if time.perf_counter() - t0 > budget or i == POINTS - 1:
                break
        return attempts / (time.perf_counter() - t0) / 1e9, i, time.perf_counter() - t0

    cores = O.threads()
    v, steps, el = timed(budget_s)
    O.set_threads(1)
    v1, steps1, el1 = timed(budget_1core_s)
    O.set_threads(cores)
    return {"value": v, "unit": "attempts/ns", "cores": cores, "kind": "oracle",
            "sample": f"{steps} temperature steps (beta_i = 3 i/300 from i = 1) of one systematic-resampling "
                      f"run with R = {Rs} replicas of the headline lattice (3D +-J L = 16, couplings seed 1), "
                      f"theta = {THETA} ({el:.1f} s)",
            "value_1_core": v1,
            "sample_1_core": f"{steps1} temperature steps of the same run on one thread ({el1:.1f} s)"}


ROWS = ("anneal", "fm2d_L64", "glass3d_L10", "resample_scaling", "batched", "learned", "combination",
        "resampling", "conditional", "scheme_errors", "rmsd", "cluster")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="only the headline (no other rows)")
    ap.add_argument("--rows", default=",".join(ROWS), help="comma-separated rows to run: " + ",".join(ROWS))
    ap.add_argument("--profile", choices=("glass3d_L16", "glass3d_L10", "fm2d_L64"),
                    help="short run for hardware counters: warmup + steps temperature steps of one run "
                         "of the workload, then a 256 MiB device-to-device copy of known size")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(this library runs one GPU; sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    if a.profile:
        profile_run(a.profile, a.steps, a.warmup)
        return
    if a.steps < 1 or a.warmup < 0:
        print("need --steps >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    r = headline_bench(a.steps, a.warmup)
    rate = philox_rate()
    value = r["attempts"] / r["elapsed"] / 1e9
    prof = profiled_counters("glass3d_L16")
    if prof:
        prof["path"] = COUNTER_PROFILES["glass3d_L16"]
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
            "workload": "3D +-J Edwards-Anderson spin glass L=16 periodic (couplings +-1 w.p. 1/2, seed 1), "
                        "R=1000000 bit-packed (64 replicas per uint64), theta=10 checkerboard Metropolis sweeps, "
                        "beta_i=3 i/300 (301 points), systematic resampling, one run",
            "dim": D, "L": L, "R": R, "theta": THETA,
            "timed_beta_range": r["beta_range"],
        },
        "sweep_attempts_per_ns": r["attempts"] / (sum(r["sweep_ms"]) * 1e-3) / 1e9,
        "resample_GB_per_s": r["res_bytes"] / (sum(r["res_ms"]) * 1e-3) / 1e9,
        "sweep_share_of_step": sum(r["sweep_ms"]) * 1e-3 / r["elapsed"],
        "roofline": sweep_roofline("k_sweep<3,true>", L ** D, r["attempts"], r["calls"], r["updates"], r["words"],
                                   r["sweep_ms"], rate, "3d_pmj", prof),
    }
    rows = [] if a.no_rows else [x for x in a.rows.split(",") if x]
    unknown = [x for x in rows if x not in ROWS]
    if unknown:
        print(f"unknown rows: {unknown}", file=sys.stderr)
        sys.exit(2)
    fns = {"anneal": lambda: anneal_row(rate), "fm2d_L64": fm2d_L64_row, "glass3d_L10": glass3d_L10_row,
           "resample_scaling": resample_scaling, "batched": batched_bench, "learned": learned_bench,
           "combination": combination_study, "resampling": resampling_study,
           "conditional": conditional_study, "scheme_errors": scheme_error_study, "rmsd": rmsd_study,
           "cluster": cluster_study}
    for name in ROWS:
        if name in rows:
            t0 = time.perf_counter()
            out[name] = fns[name]()
            out[name]["row_wall_s"] = time.perf_counter() - t0
            print(f"[bench] row {name} done ({out[name]['row_wall_s']:.1f} s)", file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
