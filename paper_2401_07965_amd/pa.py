"""Python binding of the population-annealing C ABI (include/pa.h).

Argument marshalling only: every step runs in the HIP library ``libpa.so``
built beside this file.  PyTorch provides the device workspace and the HIP
stream.  There is no fallback: without the built library every call raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpa.so")

PA_OK, PA_E_INVAL, PA_E_NOMEM, PA_E_STATE, PA_E_CAPACITY, PA_E_EXTINCT, PA_E_NONFINITE, \
    PA_E_DEVICE = range(8)
MULTINOMIAL, POISSON, NEAREST_INT, SYSTEMATIC = 0, 1, 2, 3
SCHEMES = {"multinomial": MULTINOMIAL, "poisson": POISSON, "nearest": NEAREST_INT,
           "systematic": SYSTEMATIC}


class pa_config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("L", ctypes.c_int32), ("R", ctypes.c_int64),
                ("capacity", ctypes.c_int64), ("seed", ctypes.c_uint32),
                ("run_id", ctypes.c_uint32), ("couplings", ctypes.c_void_p)]


class pa_obs(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int64), ("beta", ctypes.c_double), ("sum_E", ctypes.c_int64),
                ("sum_E2", ctypes.c_int64), ("sum_absM", ctypes.c_int64),
                ("sum_M2", ctypes.c_int64), ("sum_c2", ctypes.c_int64),
                ("families", ctypes.c_int64), ("e", ctypes.c_double), ("e2", ctypes.c_double),
                ("abs_m", ctypes.c_double), ("m2", ctypes.c_double), ("rho_t", ctypes.c_double),
                ("S_f", ctypes.c_double), ("sv", ctypes.c_double),
                ("sum_E3_hi", ctypes.c_int64), ("sum_E3_lo", ctypes.c_uint64), ("e3", ctypes.c_double),
                ("ess", ctypes.c_double), ("weighted", ctypes.c_int32), ("pad", ctypes.c_int32)]


class pa_host_state(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int64), ("step", ctypes.c_uint32), ("sweeps", ctypes.c_uint32),
                ("beta", ctypes.c_double), ("lnZ", ctypes.c_double),
                ("spins", ctypes.c_void_p), ("energy", ctypes.c_void_p),
                ("magnetization", ctypes.c_void_p), ("label", ctypes.c_void_p)]


class pa_counters(ctypes.Structure):
    _fields_ = [("philox_calls", ctypes.c_uint64), ("site_updates", ctypes.c_uint64),
                ("sweeps", ctypes.c_uint64), ("spin_attempts", ctypes.c_uint64),
                ("resamplings", ctypes.c_uint64)]


class pa_step_record(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("beta", "lnQ", "lnZ", "sv", "e", "e2", "abs_m", "m2",
                                               "rho_t", "S_f")] + \
               [(n, ctypes.c_int64) for n in ("R", "sum_E", "sum_E2", "sum_absM", "sum_M2",
                                              "sum_c2", "families")] + \
               [("status", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class pa_combined(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("lnZ", "e", "e2", "abs_m", "m2", "c", "chi", "n_eff",
                                               "beta", "c_naive", "chi_naive", "e_plain", "c_plain",
                                               "chi_plain")] + \
               [("runs", ctypes.c_int32), ("pad", ctypes.c_int32)]


class pa_mlp_norm(ctypes.Structure):
    _fields_ = [("x_mean", ctypes.c_float * 8), ("x_std", ctypes.c_float * 8),
                ("y_mean", ctypes.c_float), ("y_std", ctypes.c_float)]


MLP_PARAMS = 4801

STEP_RECORD_DTYPE = np.dtype([(n, np.float64) for n in ("beta", "lnQ", "lnZ", "sv", "e", "e2",
                                                        "abs_m", "m2", "rho_t", "S_f")] +
                             [(n, np.int64) for n in ("R", "sum_E", "sum_E2", "sum_absM", "sum_M2",
                                                      "sum_c2", "families")] +
                             [("status", np.uint32), ("pad", np.uint32)])
assert STEP_RECORD_DTYPE.itemsize == ctypes.sizeof(pa_step_record)


class PAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class CapacityError(PAError):
    pass


class ExtinctError(PAError):
    pass


class StateError(PAError):
    pass


_ERRORS = {PA_E_CAPACITY: CapacityError, PA_E_EXTINCT: ExtinctError, PA_E_STATE: StateError}
_lib = None


def lib():
    """The loaded HIP library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        v = ctypes.c_void_p
        L.pa_required_bytes.argtypes = [P(pa_config), P(ctypes.c_uint64)]
        L.pa_init.argtypes = [P(pa_config), v, ctypes.c_uint64, v, P(v)]
        L.pa_sweep.argtypes = [v, ctypes.c_int32]
        L.pa_cluster.argtypes = [v, ctypes.c_int32]
        L.pa_reweight.argtypes = [v, ctypes.c_double, P(ctypes.c_double)]
        L.pa_resample.argtypes = [v, ctypes.c_int, P(ctypes.c_int64)]
        L.pa_resample_conditional.argtypes = [v, ctypes.c_int, ctypes.c_double, P(ctypes.c_int64),
                                              P(ctypes.c_int32)]
        L.pa_log_weights.argtypes = [v, v, P(ctypes.c_int32)]
        L.pa_observables.argtypes = [v, P(pa_obs)]
        L.pa_free_energy.argtypes = [v, P(ctypes.c_double)]
        L.pa_export_state.argtypes = [v, P(pa_host_state)]
        L.pa_import_state.argtypes = [v, P(pa_host_state)]
        L.pa_overlap.argtypes = [v, v, v]
        L.pa_overlap_noalloc.argtypes = [v, v, v]
        L.pa_philox_probe.argtypes = [v, ctypes.c_int64, ctypes.c_int32, v]
        L.pa_get_counters.argtypes = [v, P(pa_counters)]
        L.pa_step_alpha.argtypes = [v, ctypes.c_double, P(ctypes.c_double)]
        L.pa_step_rule.argtypes = [v, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                   P(ctypes.c_double)]
        L.pa_batch_required_bytes.argtypes = [P(pa_config), ctypes.c_int32, ctypes.c_int32,
                                              P(ctypes.c_uint64)]
        L.pa_batch_create.argtypes = [P(pa_config), ctypes.c_int32, ctypes.c_int32, v,
                                      ctypes.c_uint64, v, P(v)]
        L.pa_batch_tune.argtypes = [v, ctypes.c_int32, ctypes.c_double, v, v]
        L.pa_batch_set_threads.argtypes = [v, ctypes.c_int32, ctypes.c_int32]
        L.pa_batch_groups.argtypes = [v, P(ctypes.c_int32), v]
        L.pa_batch_anneal.argtypes = [v, v, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                                      ctypes.c_int32]
        L.pa_batch_records.argtypes = [v, v]
        L.pa_batch_export_run.argtypes = [v, ctypes.c_int32, P(pa_host_state)]
        L.pa_batch_combine.argtypes = [v, v, ctypes.c_int32, ctypes.c_int32, v]
        L.pa_batch_overlap.argtypes = [v, ctypes.c_int32, ctypes.c_int32, v]
        L.pa_batch_destroy.argtypes = [v]
        L.pa_batch_destroy.restype = None
        L.pa_batch_last_error.argtypes = [v]
        L.pa_batch_last_error.restype = ctypes.c_char_p
        for name in ("pa_batch_required_bytes", "pa_batch_create", "pa_batch_tune", "pa_batch_set_threads",
                     "pa_batch_groups", "pa_batch_anneal", "pa_batch_records",
                     "pa_batch_export_run", "pa_batch_combine", "pa_batch_overlap"):
            getattr(L, name).restype = ctypes.c_int
        L.pa_mlp_required_bytes.argtypes = [ctypes.c_int32, P(ctypes.c_uint64)]
        L.pa_mlp_create.argtypes = [ctypes.c_int32, v, P(pa_mlp_norm), v, ctypes.c_uint64, v, P(v)]
        L.pa_mlp_set_data.argtypes = [v, v, v, ctypes.c_int32]
        L.pa_mlp_gradient.argtypes = [v, v, P(ctypes.c_double)]
        L.pa_mlp_train.argtypes = [v, ctypes.c_int32, ctypes.c_float, P(ctypes.c_double)]
        L.pa_mlp_params.argtypes = [v, v]
        L.pa_mlp_predict.argtypes = [v, v, ctypes.c_int32, v]
        L.pa_features.argtypes = [v, v]
        L.pa_step_learned.argtypes = [v, v, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int32), P(ctypes.c_double)]
        L.pa_mlp_destroy.argtypes = [v]
        L.pa_mlp_destroy.restype = None
        L.pa_mlp_last_error.argtypes = [v]
        L.pa_mlp_last_error.restype = ctypes.c_char_p
        for name in ("pa_mlp_required_bytes", "pa_mlp_create", "pa_mlp_set_data", "pa_mlp_gradient",
                     "pa_mlp_train", "pa_mlp_params", "pa_mlp_predict", "pa_features",
                     "pa_step_learned"):
            getattr(L, name).restype = ctypes.c_int
        L.pa_destroy.argtypes = [v]
        L.pa_destroy.restype = None
        L.pa_last_error.argtypes = [v]
        L.pa_last_error.restype = ctypes.c_char_p
        for name in ("pa_required_bytes", "pa_init", "pa_sweep", "pa_cluster", "pa_reweight", "pa_resample",
                     "pa_observables", "pa_free_energy", "pa_export_state", "pa_import_state",
                     "pa_overlap", "pa_overlap_noalloc", "pa_get_counters", "pa_step_alpha", "pa_step_rule",
                     "pa_philox_probe"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status, ctx):
    if status != PA_OK:
        msg = lib().pa_last_error(ctx)
        raise _ERRORS.get(status, PAError)(status, msg.decode() if msg else "")


def _check_m(status, m):
    if status != PA_OK:
        msg = lib().pa_mlp_last_error(m)
        raise _ERRORS.get(status, PAError)(status, msg.decode() if msg else "")


def _check_b(status, b):
    if status != PA_OK:
        msg = lib().pa_batch_last_error(b)
        raise _ERRORS.get(status, PAError)(status, msg.decode() if msg else "")


def make_config(dim, L, R, seed=1, run_id=0, capacity=0, couplings=None):
    """A pa_config; ``couplings`` (int8[N*dim] or None) must outlive pa_init."""
    cfg = pa_config(dim, L, int(R), int(capacity), seed & 0xFFFFFFFF, run_id & 0xFFFFFFFF, None)
    if couplings is not None:
        assert couplings.dtype == np.int8 and couplings.flags.c_contiguous
        cfg.couplings = couplings.ctypes.data
    return cfg


def pa_required_bytes(cfg):
    n = ctypes.c_uint64()
    _check(lib().pa_required_bytes(ctypes.byref(cfg), ctypes.byref(n)), None)
    return n.value


def pa_init(cfg, workspace_ptr, workspace_bytes, stream_ptr):
    ctx = ctypes.c_void_p()
    _check(lib().pa_init(ctypes.byref(cfg), workspace_ptr, workspace_bytes, stream_ptr,
                         ctypes.byref(ctx)), None)
    return ctx


def pa_sweep(ctx, theta):
    _check(lib().pa_sweep(ctx, int(theta)), ctx)


def pa_cluster(ctx, nsteps):
    _check(lib().pa_cluster(ctx, int(nsteps)), ctx)


def pa_reweight(ctx, beta_next, wait=True):
    """ln Q; with wait=False the call is deferred and returns None."""
    if not wait:
        _check(lib().pa_reweight(ctx, float(beta_next), None), ctx)
        return None
    q = ctypes.c_double()
    _check(lib().pa_reweight(ctx, float(beta_next), ctypes.byref(q)), ctx)
    return q.value


def pa_resample(ctx, scheme, wait=True):
    """New population size; with wait=False the call is deferred (a failure
    freezes the run and is raised by the next waiting call) and returns None."""
    if not wait:
        _check(lib().pa_resample(ctx, int(scheme), None), ctx)
        return None
    n = ctypes.c_int64()
    _check(lib().pa_resample(ctx, int(scheme), ctypes.byref(n)), ctx)
    return n.value


def pa_resample_conditional(ctx, scheme, kappa, wait=True):
    """(new population size, resampled?); with wait=False deferred, returns None."""
    if not wait:
        _check(lib().pa_resample_conditional(ctx, int(scheme), float(kappa), None, None), ctx)
        return None
    n = ctypes.c_int64()
    r = ctypes.c_int32()
    _check(lib().pa_resample_conditional(ctx, int(scheme), float(kappa), ctypes.byref(n),
                                         ctypes.byref(r)), ctx)
    return n.value, bool(r.value)


def pa_log_weights(ctx, R):
    """Log-weights of the R current replicas (zeros if uniform) and the weighted flag."""
    out = np.zeros(R, np.float64)
    w = ctypes.c_int32()
    _check(lib().pa_log_weights(ctx, out.ctypes.data, ctypes.byref(w)), ctx)
    return out, bool(w.value)


def pa_observables(ctx, wait=True):
    if not wait:
        _check(lib().pa_observables(ctx, None), ctx)
        return None
    o = pa_obs()
    _check(lib().pa_observables(ctx, ctypes.byref(o)), ctx)
    out = {name: getattr(o, name) for name, _ in pa_obs._fields_ if name != "pad"}
    out["sum_E3"] = (out.pop("sum_E3_hi") << 64) + out.pop("sum_E3_lo")
    out["weighted"] = bool(out["weighted"])
    return out


def pa_free_energy(ctx):
    z = ctypes.c_double()
    _check(lib().pa_free_energy(ctx, ctypes.byref(z)), ctx)
    return z.value


def pa_export_state(ctx, N, arrays=True):
    st = pa_host_state()
    _check(lib().pa_export_state(ctx, ctypes.byref(st)), ctx)
    out = dict(R=st.R, step=st.step, sweeps=st.sweeps, beta=st.beta, lnZ=st.lnZ)
    if arrays:
        R = st.R
        spins = np.zeros(((R + 63) // 64, N), np.uint64)
        E = np.zeros(R, np.int32)
        M = np.zeros(R, np.int32)
        lab = np.zeros(R, np.uint32)
        st.spins, st.energy = spins.ctypes.data, E.ctypes.data
        st.magnetization, st.label = M.ctypes.data, lab.ctypes.data
        _check(lib().pa_export_state(ctx, ctypes.byref(st)), ctx)
        out.update(spins=spins, energy=E, magnetization=M, label=lab)
    return out


def pa_import_state(ctx, R, step, sweeps, beta, lnZ, spins, energy, magnetization, label):
    spins = np.ascontiguousarray(spins, np.uint64)
    energy = np.ascontiguousarray(energy, np.int32)
    magnetization = np.ascontiguousarray(magnetization, np.int32)
    label = np.ascontiguousarray(label, np.uint32)
    st = pa_host_state(int(R), int(step), int(sweeps), float(beta), float(lnZ), spins.ctypes.data,
                       energy.ctypes.data, magnetization.ctypes.data, label.ctypes.data)
    _check(lib().pa_import_state(ctx, ctypes.byref(st)), ctx)


def philox_probe(out, iters, stream):
    """Enqueue the generator throughput probe: out is a device uint32 tensor
    (one word per thread, a multiple of 256 threads); 3 * iters Philox calls per
    thread."""
    _check(lib().pa_philox_probe(out.data_ptr(), out.numel(), int(iters), stream.cuda_stream), None)


def pa_overlap_noalloc(a, b, N):
    """pa_overlap through the allocation-free entry point (file-scope device histogram)."""
    h = np.zeros(N + 1, np.int64)
    _check(lib().pa_overlap_noalloc(a, b, h.ctypes.data), a)
    return h


def pa_overlap(a, b, N):
    h = np.zeros(N + 1, np.int64)
    _check(lib().pa_overlap(a, b, h.ctypes.data), a)
    return h


def pa_step_alpha(ctx, dbeta):
    a = ctypes.c_double()
    _check(lib().pa_step_alpha(ctx, float(dbeta), ctypes.byref(a)), ctx)
    return a.value


def pa_step_rule(ctx, alpha_star, dbeta_max, iterations=60):
    d = ctypes.c_double()
    _check(lib().pa_step_rule(ctx, float(alpha_star), float(dbeta_max), int(iterations),
                              ctypes.byref(d)), ctx)
    return d.value


def pa_get_counters(ctx):
    c = pa_counters()
    _check(lib().pa_get_counters(ctx, ctypes.byref(c)), ctx)
    return {name: getattr(c, name) for name, _ in pa_counters._fields_}


def pa_destroy(ctx):
    lib().pa_destroy(ctx)


# ------------------------------------------------------------------ conveniences
def unpack_spins(words, R):
    """[W][N] uint64 words -> int8 spins [R][N] (+1/-1), replica 64w+b = bit b."""
    W, N = words.shape
    bits = np.unpackbits(np.ascontiguousarray(words).view(np.uint8).reshape(W, N, 8),
                         axis=2, bitorder="little")  # [W, N, 64]
    bits = bits.transpose(0, 2, 1).reshape(W * 64, N)[:R]
    return (1 - 2 * bits.astype(np.int8)).astype(np.int8)


def pack_spins(spins):
    """int8 spins [R][N] (+1/-1) -> [ceil(R/64)][N] uint64 words."""
    R, N = spins.shape
    W = (R + 63) // 64
    bits = np.zeros((W * 64, N), np.uint8)
    bits[:R] = (spins < 0)
    by = np.packbits(bits.reshape(W, 64, N).transpose(0, 2, 1), axis=2, bitorder="little")
    return np.ascontiguousarray(by).view(np.uint64).reshape(W, N)


class PARun:
    """One PA run on the GPU: a torch-owned workspace, a stream and a context."""

    def __init__(self, dim, L, R, seed=1, run_id=0, capacity=0, couplings=None, device=None,
                 stream=None):
        import torch
        self.dim, self.L, self.R = dim, L, int(R)
        self.N = L ** dim
        self.couplings = None if couplings is None else np.ascontiguousarray(couplings, np.int8)
        cfg = make_config(dim, L, R, seed, run_id, capacity, self.couplings)
        nbytes = pa_required_bytes(cfg)
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace not 256-byte aligned")
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self.ctx = pa_init(cfg, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)

    def reweight(self, beta_next, wait=True):
        return pa_reweight(self.ctx, beta_next, wait)

    def resample(self, scheme, wait=True):
        return pa_resample(self.ctx, SCHEMES.get(scheme, scheme), wait)

    def resample_conditional(self, scheme, kappa, wait=True):
        return pa_resample_conditional(self.ctx, SCHEMES.get(scheme, scheme), kappa, wait)

    def log_weights(self):
        """(log-weights of the current replicas, weighted flag)."""
        R = pa_export_state(self.ctx, self.N, arrays=False)["R"]
        return pa_log_weights(self.ctx, R)

    def sweep(self, theta):
        pa_sweep(self.ctx, theta)

    def cluster(self, nsteps):
        """nsteps Wolff single-cluster updates of every replica (the
        cluster-update driver); enqueued, like sweep."""
        pa_cluster(self.ctx, nsteps)

    def observables(self, wait=True):
        return pa_observables(self.ctx, wait)

    def free_energy(self):
        return pa_free_energy(self.ctx)

    def export(self, arrays=True):
        return pa_export_state(self.ctx, self.N, arrays)

    def import_state(self, **kw):
        pa_import_state(self.ctx, **kw)

    def overlap(self, other):
        return pa_overlap(self.ctx, other.ctx, self.N)

    def overlap_noalloc(self, other):
        return pa_overlap_noalloc(self.ctx, other.ctx, self.N)

    def step_alpha(self, dbeta):
        return pa_step_alpha(self.ctx, dbeta)

    def step_rule(self, alpha_star, dbeta_max, iterations=60):
        return pa_step_rule(self.ctx, alpha_star, dbeta_max, iterations)

    def counters(self):
        return pa_get_counters(self.ctx)

    def features(self):
        out = np.zeros(8, np.float32)
        _check(lib().pa_features(self.ctx, out.ctypes.data), self.ctx)
        return out

    def step_learned(self, mlp, alpha_star, dbeta_max, iterations=60, bracket=1.0, refine=0, proposal=False):
        """(dbeta, fallback) of pa_step_learned; with proposal=True also the
        model's clamped proposal."""
        d = ctypes.c_double()
        fb = ctypes.c_int32()
        c = ctypes.c_double()
        _check(lib().pa_step_learned(self.ctx, mlp.h, float(alpha_star), float(dbeta_max), int(iterations),
                                     float(bracket), int(refine), ctypes.byref(d), ctypes.byref(fb),
                                     ctypes.byref(c)), self.ctx)
        if proposal:
            return d.value, bool(fb.value), c.value
        return d.value, bool(fb.value)

    def close(self):
        if self.ctx is not None:
            pa_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PABatch:
    """Many independent runs annealed together (one workspace, one stream).

    ``configs``: list of dicts with dim, L, R and optional seed, run_id,
    capacity, couplings (int8[N*dim])."""

    def __init__(self, configs, max_points, device=None, stream=None):
        import torch
        self.n = len(configs)
        self._coup = [None if c.get("couplings") is None else
                      np.ascontiguousarray(c["couplings"], np.int8) for c in configs]
        arr = (pa_config * self.n)()
        for k, c in enumerate(configs):
            arr[k] = make_config(c["dim"], c["L"], c["R"], c.get("seed", 1), c.get("run_id", 0),
                                 c.get("capacity", 0), self._coup[k])
        self._cfgs = arr
        self.N = [c["L"] ** c["dim"] for c in configs]
        self.max_points = int(max_points)
        nb = ctypes.c_uint64()
        _check_b(lib().pa_batch_required_bytes(arr, self.n, self.max_points, ctypes.byref(nb)), None)
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        # graph capture needs a stream of its own (default priority)
        self.stream = torch.cuda.Stream(self.device) if stream is None else stream
        torch.cuda.synchronize(self.device)
        h = ctypes.c_void_p()
        _check_b(lib().pa_batch_create(arr, self.n, self.max_points, self.workspace.data_ptr(),
                                       nb.value, self.stream.cuda_stream, ctypes.byref(h)), None)
        self.h = h
        self.npoints = 0

    def groups(self):
        ng = ctypes.c_int32()
        t = np.zeros(16, np.int32)
        _check_b(lib().pa_batch_groups(self.h, ctypes.byref(ng), t.ctypes.data), self.h)
        return t[:ng.value].tolist()

    def tune(self, theta=10, beta=1.0, times=False):
        """Autotunes each group's sweep workgroup size with theta sweeps at the
        thresholds of beta; returns the chosen sizes (and, with times=True, a
        dict {group: {threads: ms}} of every candidate's time)."""
        t = np.zeros(16, np.int32)
        ms = np.zeros(16 * 12, np.float32)
        _check_b(lib().pa_batch_tune(self.h, int(theta), float(beta), t.ctypes.data, ms.ctypes.data), self.h)
        chosen = self.groups()
        if not times:
            return chosen
        tab = {g: {64 * (k + 1): float(ms[g * 12 + k]) for k in range(12) if ms[g * 12 + k] >= 0}
               for g in range(len(chosen))}
        return chosen, tab

    def set_threads(self, group, threads):
        _check_b(lib().pa_batch_set_threads(self.h, int(group), int(threads)), self.h)

    def anneal(self, betas, theta, scheme, use_graph=True):
        b = np.ascontiguousarray(betas, np.float64)
        _check_b(lib().pa_batch_anneal(self.h, b.ctypes.data, len(b), int(theta),
                                       SCHEMES.get(scheme, scheme), 1 if use_graph else 0), self.h)
        self.npoints = len(b)

    def records(self):
        out = np.zeros((self.n, self.npoints), STEP_RECORD_DTYPE)
        _check_b(lib().pa_batch_records(self.h, out.ctypes.data), self.h)
        return out

    def export_run(self, m):
        st = pa_host_state()
        _check_b(lib().pa_batch_export_run(self.h, m, ctypes.byref(st)), self.h)
        R, N = st.R, self.N[m]
        spins = np.zeros(((R + 63) // 64, N), np.uint64)
        E = np.zeros(R, np.int32)
        M = np.zeros(R, np.int32)
        lab = np.zeros(R, np.uint32)
        st.spins, st.energy = spins.ctypes.data, E.ctypes.data
        st.magnetization, st.label = M.ctypes.data, lab.ctypes.data
        _check_b(lib().pa_batch_export_run(self.h, m, ctypes.byref(st)), self.h)
        return dict(R=R, step=st.step, sweeps=st.sweeps, beta=st.beta, lnZ=st.lnZ, spins=spins,
                    energy=E, magnetization=M, label=lab)

    def overlap(self, a, b):
        """Overlap histogram (int64[N + 1]) between runs a and b (pa_batch_overlap)."""
        h = np.zeros(self.N[a] + 1, np.int64)
        _check_b(lib().pa_batch_overlap(self.h, int(a), int(b), h.ctypes.data), self.h)
        return h

    def combine(self, group_of_run, ngroups, point):
        g = np.ascontiguousarray(group_of_run, np.int32)
        out = (pa_combined * ngroups)()
        _check_b(lib().pa_batch_combine(self.h, g.ctypes.data, int(ngroups), int(point),
                                        ctypes.cast(out, ctypes.c_void_p)), self.h)
        return [{n: getattr(o, n) for n, _ in pa_combined._fields_ if n != "pad"} for o in out]

    def close(self):
        if self.h is not None:
            lib().pa_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PAMlp:
    """The learned temperature-step model on the GPU (train, predict)."""

    def __init__(self, params, x_mean, x_std, y_mean, y_std, max_samples, device=None,
                 stream=None):
        import torch
        self.params0 = np.ascontiguousarray(params, np.float32)
        assert self.params0.shape == (MLP_PARAMS,)
        nm = pa_mlp_norm()
        for k in range(8):
            nm.x_mean[k], nm.x_std[k] = float(x_mean[k]), float(x_std[k])
        nm.y_mean, nm.y_std = float(y_mean), float(y_std)
        self.norm = nm
        nb = ctypes.c_uint64()
        _check_m(lib().pa_mlp_required_bytes(int(max_samples), ctypes.byref(nb)), None)
        self.device = torch.device("cuda", 0) if device is None else torch.device(device)
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = ctypes.c_void_p()
        _check_m(lib().pa_mlp_create(int(max_samples), self.params0.ctypes.data, ctypes.byref(nm),
                                     self.workspace.data_ptr(), nb.value, self.stream.cuda_stream,
                                     ctypes.byref(h)), None)
        self.h = h

    def set_data(self, X, y):
        X = np.ascontiguousarray(X, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        _check_m(lib().pa_mlp_set_data(self.h, X.ctypes.data, y.ctypes.data, len(y)), self.h)

    def gradient(self):
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = ctypes.c_double()
        _check_m(lib().pa_mlp_gradient(self.h, g.ctypes.data, ctypes.byref(loss)), self.h)
        return g, loss.value

    def train(self, epochs, lr):
        loss = ctypes.c_double()
        _check_m(lib().pa_mlp_train(self.h, int(epochs), float(lr), ctypes.byref(loss)), self.h)
        return loss.value

    def params(self):
        p = np.zeros(MLP_PARAMS, np.float32)
        _check_m(lib().pa_mlp_params(self.h, p.ctypes.data), self.h)
        return p

    def predict(self, X):
        X = np.ascontiguousarray(X, np.float32)
        out = np.zeros(len(X), np.float32)
        _check_m(lib().pa_mlp_predict(self.h, X.ctypes.data, len(X), out.ctypes.data), self.h)
        return out

    def close(self):
        if self.h is not None:
            lib().pa_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
