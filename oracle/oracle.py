"""CPU oracle for the population-annealing hot path (Python side).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It drives ``pa_oracle.c`` (plain C:
Philox, the deterministic exponential, initial sampling, Metropolis sweeps,
Q and the resampling counts) and adds the plain population averages of
step 4 of the algorithm (Sec. 2), the family statistics of Eq. (6), the
sampling variance of Eq. (5) and the free energy of Eq. (7).

The step cycle follows the enumerated algorithm of Sec. 2: ``reweight`` to the
next inverse temperature (step 2, Q of Eq. (1)), ``resample`` (step 2, Sec. 3),
``sweep`` (step 3), ``observables`` (step 4).  ``resample_conditional``
resamples only when the weights' effective sample size is small (the remark
of Sec. 3 that resampling need not happen at every step); a kept population
carries importance weights, which reweighting and the averages then use.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

_LIB = None

MULTINOMIAL, POISSON, NEAREST_INT, SYSTEMATIC = 0, 1, 2, 3
SCHEMES = {"multinomial": MULTINOMIAL, "poisson": POISSON, "nearest": NEAREST_INT,
           "systematic": SYSTEMATIC}
FIXED_SIZE = (MULTINOMIAL, SYSTEMATIC)

_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_c = ctypes


def lib():
    """Load (building first if needed) the oracle's C library."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_philox.argtypes = [_c.c_uint32, _c.c_uint32, _u32p, _u32p]
        L.orc_philox.restype = None
        L.orc_exp.argtypes = [_c.c_double]
        L.orc_exp.restype = _c.c_double
        L.orc_threshold.argtypes = [_c.c_double, _c.c_int]
        L.orc_threshold.restype = _c.c_uint64
        L.orc_energy.argtypes = [_c.c_int, _c.c_int, _i8p, _i8p]
        L.orc_energy.restype = _c.c_int64
        L.orc_init.argtypes = [_c.c_int, _c.c_int, _c.c_int64, _i64p, _c.c_uint32, _c.c_uint32,
                               _i8p, _i8p, _i32p, _u32p]
        L.orc_init.restype = None
        L.orc_sweep.argtypes = [_c.c_int, _c.c_int, _i8p, _c.c_int64, _i64p, _i8p, _i32p,
                                _c.c_uint32, _c.c_uint32, _c.c_uint32, _c.c_uint32, _c.c_int32,
                                _c.c_double, _c.POINTER(_c.c_uint64)]
        L.orc_sweep.restype = None
        L.orc_wolff_threshold.argtypes = [_c.c_double]
        L.orc_wolff_threshold.restype = _c.c_uint64
        L.orc_wolff.argtypes = [_c.c_int, _c.c_int, _i8p, _c.c_int64, _i64p, _i8p, _i32p,
                                _c.c_uint32, _c.c_uint32, _c.c_uint32, _c.c_uint32, _c.c_int32,
                                _c.c_double, _i64p]
        L.orc_wolff.restype = None
        L.orc_reweight.argtypes = [_c.c_int64, _i32p, _c.c_double, _c.POINTER(_c.c_double), _u64p,
                                   _c.POINTER(_c.c_uint64)]
        L.orc_reweight.restype = None
        L.orc_counts.argtypes = [_c.c_int, _c.c_int64, _c.c_int64, _u64p, _c.c_uint64, _c.c_uint32,
                                 _c.c_uint32, _c.c_uint32, _u32p]
        L.orc_counts.restype = _c.c_int
        L.orc_apply.argtypes = [_c.c_int64, _c.c_int64, _u32p, _i8p, _i32p, _u32p, _i8p, _i32p,
                                _u32p]
        L.orc_apply.restype = None
        _f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        L.orc_exp_array.argtypes = [_c.c_int64, _f64p, _f64p]
        L.orc_exp_array.restype = None
        L.orc_threads.argtypes = []
        L.orc_threads.restype = _c.c_int
        L.orc_set_threads.argtypes = [_c.c_int]
        L.orc_set_threads.restype = None
        _LIB = L
    return _LIB


def threads():
    """OpenMP threads the oracle's sweeps run on."""
    return int(lib().orc_threads())


def set_threads(n):
    """Sets the OpenMP threads of the oracle's sweeps (for timing on fewer cores)."""
    lib().orc_set_threads(int(n))


# --------------------------------------------------------------------------- primitives
def philox(k0, k1, ctr):
    """Philox4x32-10 of a 4-word counter under key (k0, k1)."""
    out = np.zeros(4, np.uint32)
    lib().orc_philox(k0 & 0xFFFFFFFF, k1 & 0xFFFFFFFF, np.asarray(ctr, np.uint32), out)
    return out


def pa_exp(x):
    """Deterministic exp used wherever exp() decides something."""
    return lib().orc_exp(float(x))


def pa_exp_array(x):
    """pa_exp elementwise."""
    x = np.ascontiguousarray(x, np.float64)
    out = np.empty_like(x)
    lib().orc_exp_array(len(x), x, out)
    return out


def threshold(beta, dE):
    """Metropolis acceptance threshold T(dE) = min(2^32, floor(2^32 pa_exp(-beta dE)))."""
    return int(lib().orc_threshold(float(beta), int(dE)))


def n_sites(d, L):
    return L ** d


def ferromagnet(d, L):
    """Couplings J = +1 on every bond, layout J[s*d + mu]."""
    return np.ones(n_sites(d, L) * d, np.int8)


def energy(d, L, J, spins):
    """H of Eq. (4) (with bond-wise J) for one replica's int8 spins."""
    return int(lib().orc_energy(d, L, np.ascontiguousarray(J, np.int8),
                                np.ascontiguousarray(spins, np.int8)))


def init_rows(d, L, rows, seed, run_id, J):
    """Exact beta_0 = 0 samples for the replicas listed in ``rows``."""
    rows = np.ascontiguousarray(rows, np.int64)
    N = n_sites(d, L)
    spins = np.zeros((len(rows), N), np.int8)
    E = np.zeros(len(rows), np.int32)
    label = np.zeros(len(rows), np.uint32)
    lib().orc_init(d, L, len(rows), rows, seed, run_id, np.ascontiguousarray(J, np.int8), spins, E,
                   label)
    return spins, E, label


def sweep_rows(d, L, J, rows, spins, E, seed, run_id, step, t0, theta, beta):
    """theta Metropolis sweeps (in place) of the replicas listed in ``rows``.
    Returns the plane pairs (Philox evaluations) deciding them needed: per
    word-site, pairs up to the one where its slowest drawing replica decides."""
    rows = np.ascontiguousarray(rows, np.int64)
    assert np.all(np.diff(rows) > 0) if len(rows) > 1 else True
    assert spins.dtype == np.int8 and spins.flags.c_contiguous and E.dtype == np.int32
    calls = ctypes.c_uint64()
    lib().orc_sweep(d, L, np.ascontiguousarray(J, np.int8), len(rows), rows, spins, E, seed,
                    run_id, step, t0, theta, float(beta), ctypes.byref(calls))
    return calls.value


def wolff_rows(d, L, J, rows, spins, E, seed, run_id, step, t0, nsteps, beta):
    """nsteps Wolff single-cluster updates (in place) of the replicas listed in
    ``rows`` (the cluster-update driver; see orc_wolff for the random-number
    layout).  Returns the cluster sizes, [len(rows)][nsteps]."""
    rows = np.ascontiguousarray(rows, np.int64)
    assert spins.dtype == np.int8 and spins.flags.c_contiguous and E.dtype == np.int32
    sizes = np.zeros((len(rows), max(int(nsteps), 0)), np.int64)
    lib().orc_wolff(d, L, np.ascontiguousarray(J, np.int8), len(rows), rows, spins, E, seed, run_id,
                    step, t0, nsteps, float(beta), sizes.reshape(-1) if sizes.size else
                    np.zeros(1, np.int64))
    return sizes


def wolff_threshold(beta):
    """T_p = min(2^32, floor(2^32 (1 - pa_exp(-2 beta)))): a bond joins the
    cluster iff it is satisfied and the replica's uniform u < T_p."""
    return int(lib().orc_wolff_threshold(float(beta)))


def reweight(E, dbeta):
    """ln Q of Eq. (1), the integer weights W_j and their sum S."""
    E = np.ascontiguousarray(E, np.int32)
    W = np.zeros(len(E), np.uint64)
    lnQ = ctypes.c_double()
    S = ctypes.c_uint64()
    lib().orc_reweight(len(E), E, float(dbeta), ctypes.byref(lnQ), W, ctypes.byref(S))
    return lnQ.value, W, S.value


def counts(scheme, W, S, R_target, seed, run_id, step):
    """Copy numbers r_j of one resampling step (Sec. 3)."""
    W = np.ascontiguousarray(W, np.uint64)
    r = np.zeros(len(W), np.uint32)
    rc = lib().orc_counts(scheme, len(W), R_target, W, S, seed, run_id, step, r)
    if rc != 0:
        raise ValueError("orc_counts rejected its arguments")
    return r


def apply_counts(N, r, spins, E, label):
    """New population: r_j copies of replica j, in ascending j."""
    Rn = int(r.sum(dtype=np.int64))
    so = np.zeros((Rn, N), np.int8)
    eo = np.zeros(Rn, np.int32)
    lo = np.zeros(Rn, np.uint32)
    lib().orc_apply(N, len(r), np.ascontiguousarray(r, np.uint32), spins, E, label, so, eo, lo)
    return so, eo, lo


def tau_hat(W, S, R_target):
    """tauhat_j = R W_j / S as doubles (Eq. (3) with the quantised weights)."""
    return (W.astype(np.float64) / float(S)) * float(R_target)


# --------------------------------------------------------------------------- weighted populations
# Sec. 3 notes that resampling need not happen at every temperature step: the
# population can be kept, with importance weights, until their variance grows
# too large.  A kept replica j carries a log-weight lw_j <= 0 (largest 0); its
# weight at the next inverse temperature is exp(lw_j - dbeta E_j), so Q of
# Eq. (1) becomes the ratio of weighted sums and the resampling draws with
# tauhat_j proportional to that weight.

def weighted_reweight(E, lw, dbeta):
    """Reweighting of a population with log-weights ``lw`` (zeros: uniform).

    With x_j = lw_j + (-(dbeta (E_j - E_min))) and m = min_j |x_j| (every x_j is
    <= 0, so max_j x_j = -m):
      lnQ = ln sum_j exp(lw_j - dbeta E_j) - ln sum_j exp(lw_j)
          = -dbeta E_min - m + ln sum_j exp(x_j + m) - ln sum_j exp(lw_j),
      W_j = floor(2^40 pa_exp(x_j + m)),  S = sum_j W_j,
    and the log-weights the population keeps if it is not resampled are
    x_j + m.  With lw = 0 the integer weights are those of ``reweight``.
    """
    E = np.asarray(E, np.int64)
    lw = np.asarray(lw, np.float64)
    emin = int(E.min())
    x = lw + (-(float(dbeta) * (E - emin).astype(np.float64)))
    m = float(np.abs(x).min())
    y = x + m
    W = np.floor(np.ldexp(pa_exp_array(y), 40)).astype(np.uint64)
    lnQ = (-float(dbeta) * emin - m + math.log(float(np.sum(np.exp(y))))
           - math.log(float(np.sum(np.exp(lw)))))
    return dict(lnQ=lnQ, W=W, S=int(W.sum(dtype=np.uint64)), lw_next=y)


KAPPA_ONE = 65536  # the ESS fraction kappa in units of 2^-16


def kappa_units(kappa):
    """kappa in [0, 1] as an integer count of 2^-16 (nearest, halves up)."""
    if not 0.0 <= kappa <= 1.0:
        raise ValueError("kappa must lie in [0, 1]")
    return int(math.floor(kappa * KAPPA_ONE + 0.5))


def ess_resamples(W, kq):
    """Whether the population resamples: its effective sample size
    ESS = (sum_j W_j)^2 / sum_j W_j^2 lies below kappa R, decided exactly in
    integers as 2^16 S^2 < kq R sum_j W_j^2 (R = len(W), kq = kappa 2^16)."""
    S = sum(int(w) for w in W)
    Q2 = sum(int(w) * int(w) for w in W)
    return KAPPA_ONE * S * S < int(kq) * len(W) * Q2, S, Q2


def ess(W):
    """ESS = S^2 / sum W^2 as a double."""
    S = sum(int(w) for w in W)
    Q2 = sum(int(w) * int(w) for w in W)
    return S * S / Q2


# --------------------------------------------------------------------------- one PA run
class PAError(Exception):
    pass


class CapacityError(PAError):
    pass


class ExtinctError(PAError):
    pass


class OracleRun:
    """One population-annealing run, step by step (Sec. 2).

    State: replicas' int8 spins (row = replica), energies, family labels, the
    current inverse temperature, the step index i, the sweep counter t within
    the step and ln Z_hat = ln Z_0 + sum_k ln Q_k (Eq. (7)).  After a step that
    kept its population (``resample_conditional``) the replicas carry
    log-weights ``lw`` (None: uniform).
    """

    def __init__(self, d, L, R, seed=1, run_id=0, J=None, capacity=None):
        if d not in (2, 3) or L < 2 or L % 2 or R < 1:
            raise ValueError("need d in {2,3}, even L >= 2, R >= 1")
        self.d, self.L, self.R = d, L, int(R)
        self.N = n_sites(d, L)
        self.seed, self.run_id = seed, run_id
        self.J = ferromagnet(d, L) if J is None else np.ascontiguousarray(J, np.int8)
        self.capacity = int(capacity) if capacity is not None else default_capacity(R)
        self.spins, self.E, self.label = init_rows(d, L, np.arange(R), seed, run_id, self.J)
        self.beta = 0.0
        self.step = 0
        self.t = 0
        self.R0 = int(R)
        # ln Z_0 at beta_0 = 0 is N ln 2 (2^N states)
        self.lnZ = float(self.N) * math.log(2.0)
        self.pending = None
        self.last_sv = 0.0
        self.last_counts = None
        self.lw = None
        self.resamplings = 0
        self.philox_calls = 0  # plane pairs the sweeps needed (work count)

    @property
    def Rcur(self):
        return len(self.E)

    def import_state(self, spins, E, label):
        self.spins = np.ascontiguousarray(spins, np.int8).copy()
        self.E = np.ascontiguousarray(E, np.int32).copy()
        self.label = np.ascontiguousarray(label, np.uint32).copy()
        self.lw = None

    def log_weights(self):
        """Per-replica log-weights (zeros for a uniform population)."""
        return np.zeros(self.Rcur) if self.lw is None else self.lw.copy()

    def reweight(self, beta_next):
        if beta_next < self.beta:
            raise ValueError("beta must not decrease")
        dbeta = float(beta_next) - self.beta
        if self.lw is None:
            lnQ, W, S = reweight(self.E, dbeta)
            self.pending = dict(beta=float(beta_next), lnQ=lnQ, W=W, S=S, dbeta=dbeta)
        else:
            p = weighted_reweight(self.E, self.lw, dbeta)
            lnQ = p["lnQ"]
            self.pending = dict(beta=float(beta_next), lnQ=lnQ, W=p["W"], S=p["S"], dbeta=dbeta,
                                lw_next=p["lw_next"])
        return lnQ

    def resample_conditional(self, scheme, kappa):
        """Resample (as ``resample``) only if the effective sample size of the
        step's weights is below kappa R_cur; otherwise keep the population with
        its new log-weights, and advance beta, the step and ln Z_hat as a
        resampling would.  Returns (R, resampled)."""
        if self.pending is None:
            raise PAError("resample before reweight")
        go, _, _ = ess_resamples(self.pending["W"], kappa_units(kappa))
        if go:
            return self.resample(scheme), True
        p = self.pending
        lw_next = p.get("lw_next")
        if lw_next is None:
            lw_next = weighted_reweight(self.E, np.zeros(self.Rcur), p["dbeta"])["lw_next"]
        if not math.isfinite(p["lnQ"]):
            raise PAError("ln Q is not finite")
        self.lw = lw_next
        self.last_sv = 0.0
        self.last_counts = None
        self.lnZ += p["lnQ"]
        self.beta = p["beta"]
        self.step += 1
        self.t = 0
        self.pending = None
        return self.Rcur, False

    def resample(self, scheme):
        if self.pending is None:
            raise PAError("resample before reweight")
        p = self.pending
        step = self.step + 1
        r = counts(scheme, p["W"], p["S"], self.R, self.seed, self.run_id, step)
        Rn = int(r.sum(dtype=np.int64))
        if Rn > self.capacity:
            raise CapacityError(Rn)
        if Rn == 0:
            raise ExtinctError()
        tau = tau_hat(p["W"], p["S"], self.R)
        self.last_sv = float(np.mean((r.astype(np.float64) - tau) ** 2))
        self.last_counts = r
        self.spins, self.E, self.label = apply_counts(self.N, r, self.spins, self.E, self.label)
        self.lw = None
        self.resamplings += 1
        self.lnZ += p["lnQ"]
        self.beta = p["beta"]
        self.step = step
        self.t = 0
        self.pending = None
        return Rn

    def sweep(self, theta):
        self.philox_calls += sweep_rows(self.d, self.L, self.J, np.arange(self.Rcur), self.spins, self.E,
                                        self.seed, self.run_id, self.step, self.t, theta, self.beta)
        self.t += theta

    def cluster(self, nsteps):
        """nsteps Wolff updates at the current beta (the update counter t is
        shared with the sweeps); returns the cluster sizes [Rcur][nsteps]."""
        sizes = wolff_rows(self.d, self.L, self.J, np.arange(self.Rcur), self.spins, self.E, self.seed,
                           self.run_id, self.step, self.t, nsteps, self.beta)
        self.t += nsteps
        return sizes

    def magnetization(self):
        return self.spins.astype(np.int64).sum(axis=1)

    def observables(self):
        return population_observables(self.N, self.E, self.magnetization(), self.label, self.R0,
                                      self.last_sv, self.lw)

    def free_energy(self):
        """ln Z_hat = -beta_i F_hat_i, Eq. (7)."""
        return self.lnZ


def default_capacity(R):
    """R + 8 ceil(sqrt R) + 64, rounded up to a multiple of 64 (fluctuations ~ sqrt R, Sec. 3)."""
    R = int(R)
    ceil_sqrt = math.isqrt(R - 1) + 1
    c = R + 8 * ceil_sqrt + 64
    return (c + 63) // 64 * 64


def population_observables(N, E, M, label, R0, sv, lw=None):
    """Plain population averages (step 4 of Sec. 2) and the family statistics.

    Exact integer sums, then: e = <E>/N, e2 = <E^2>/N^2, e3 = <E^3>/N^3, |m|, m^2, the family
    measure rho_t = R sum_k n_k^2 of Eq. (6) with n_k = c_k / R (so
    rho_t = sum_k c_k^2 / R), the family entropy S_f = -sum_k n_k ln n_k and
    the sampling variance of the last resampling, Eq. (5).

    A weighted population (log-weights ``lw``) reports the weighted averages
    sum_j w_j O_j / sum_j w_j, w_j = exp(lw_j), in e, e2, e3, abs_m and m2, and
    its effective size ess = (sum w)^2 / sum w^2; the integer sums and the
    family statistics stay those of the members.
    """
    R = len(E)
    E = np.asarray(E, np.int64)
    M = np.asarray(M, np.int64)
    sumE = int(E.sum())
    sumE2 = int((E * E).sum())
    # |E^3| < 2^47; chunks of 2^15 keep every partial sum inside int64
    E3 = E * E * E
    sumE3 = sum(int(E3[k:k + 32768].sum()) for k in range(0, R, 32768))
    sumAbsM = int(np.abs(M).sum())
    sumM2 = int((M * M).sum())
    c = np.bincount(np.asarray(label, np.int64), minlength=R0).astype(np.int64)
    sumC2 = int((c * c).sum())
    cpos = c[c > 0].astype(np.float64)
    rho_t = sumC2 / R
    S_f = math.log(R) - float(np.sum(cpos * np.log(cpos))) / R
    Ef = E.astype(np.float64)
    mean = sumE / R
    var = sumE2 / R - mean * mean
    m3 = float(np.mean((Ef - mean) ** 3))
    skew = m3 / var ** 1.5 if var > 0 else 0.0
    out = dict(R=R, sumE=sumE, sumE2=sumE2, sumE3=sumE3, sumAbsM=sumAbsM, sumM2=sumM2, sumC2=sumC2,
               families=int((c > 0).sum()), e=sumE / (N * R), e2=sumE2 / (N * N * R),
               e3=sumE3 / (N * N * N * R),
               abs_m=sumAbsM / (N * R), m2=sumM2 / (N * N * R), rho_t=rho_t, S_f=S_f, sv=sv,
               E_mean=mean, E_var=var, E_skew=skew, weighted=False, ess=float(R))
    if lw is not None:
        w = np.exp(np.asarray(lw, np.float64))
        sw = float(w.sum())
        Mf = M.astype(np.float64)

        def avg(v):
            return float(np.sum(w * v)) / sw
        out.update(e=avg(Ef) / N, e2=avg(Ef * Ef) / (N * N), e3=avg(Ef * Ef * Ef) / (N * N * N),
                   abs_m=avg(np.abs(Mf)) / N, m2=avg(Mf * Mf) / (N * N), weighted=True,
                   ess=sw * sw / float(np.sum(w * w)))
    return out


def overlap_histogram(words_a, words_b, R_a, R_b, N):
    """Overlap distribution between two populations of the same lattice in
    the packed layout (replica 64w + b is bit b of word [w][s], bit 1 for
    sigma = -1): replica d of a paired with replica d of b for
    d < min(R_a, R_b); entry k counts the pairs whose spins agree on k sites,
    i.e. q = (2k - N) / N = (1/N) sum_s sigma_s^a sigma_s^b (the overlap of
    Figs. 6-7).  Counted column by column from the unpacked bits."""
    R = min(int(R_a), int(R_b))
    hist = np.zeros(N + 1, np.int64)
    W = (R + 63) // 64
    for w0 in range(0, W, 256):
        w1 = min(W, w0 + 256)
        x = np.ascontiguousarray(words_a[w0:w1] ^ words_b[w0:w1])  # (C, N) uint64
        bits = np.unpackbits(x.view(np.uint8).reshape(x.shape[0], N, 8), axis=2, bitorder="little")
        differ = bits.reshape(x.shape[0], N, 64).sum(axis=1, dtype=np.int64)  # (C, 64) per replica
        same = (N - differ).reshape(-1)
        rows = 64 * w0 + np.arange(same.size)
        hist += np.bincount(same[rows < R], minlength=N + 1)
    return hist
