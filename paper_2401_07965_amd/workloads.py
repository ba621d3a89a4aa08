"""Seeded synthetic inputs of the benchmark and test workloads.

Only inputs live here (lattice shapes, couplings, population sizes, seeds,
temperature schedules); none of the method's arithmetic.  Both the tests
(which feed the CPU oracle and the HIP library from them) and bench.py use
these generators.
"""
import numpy as np


def linear_schedule(beta_f, points):
    """beta_i = i beta_f / (points - 1), i = 0..points-1 (both ends included)."""
    return [i * beta_f / (points - 1) for i in range(points)]


def pm_j_couplings(d, L, seed):
    """+-J Edwards-Anderson couplings, J = -1 with probability 1/2, int8[N*d] at s*d + mu."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random(L ** d * d) < 0.5, -1, 1).astype(np.int8)


def uneven_batch(samples=16, runs_per_sample=16, seed0=1000, R_lo=1e3, R_hi=1e5,
                 sizes=(8, 12, 16, 24)):
    """Many independent +-J runs of uneven size: per disorder sample s a lattice
    dimension d in {2, 3} and side L drawn from the sample's generator
    (seed0 + s), its own couplings, and per run R = round(10^u), u uniform in
    [log10 R_lo, log10 R_hi].  Returns (configs, group_of_run)."""
    cfgs, groups = [], []
    lo, hi = np.log10(R_lo), np.log10(R_hi)
    k = 0
    for s in range(samples):
        rng = np.random.default_rng(seed0 + s)
        d = int(rng.choice([2, 3]))
        L = int(rng.choice(list(sizes)))
        J = np.where(rng.random(L ** d * d) < 0.5, -1, 1).astype(np.int8)
        for _ in range(runs_per_sample):
            R = int(round(10 ** rng.uniform(lo, hi)))
            cfgs.append(dict(dim=d, L=L, R=R, seed=1, run_id=k, couplings=J))
            groups.append(s)
            k += 1
    return cfgs, groups


def mlp_initial_parameters(seed, hidden=64, inputs=8):
    """Seeded starting point of the step model's training: float32 vector in
    the layout W1[h][8], b1[h], W2[h][h], b2[h], W3[h], b3, weights uniform in
    +-1/sqrt(fan in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, (hidden, inputs)) / np.sqrt(inputs), np.zeros(hidden),
             rng.uniform(-1, 1, (hidden, hidden)) / np.sqrt(hidden), np.zeros(hidden),
             rng.uniform(-1, 1, hidden) / np.sqrt(hidden), np.zeros(1)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
