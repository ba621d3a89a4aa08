"""Run descriptions in JSON, and a linear-schedule anneal that writes one
JSON line per temperature step.

A run file (``paper_2401_07965_amd/runs/*.json``) holds::

    {"workload": "<what it is>", "dim": 2 | 3, "L": even int >= 2, "R": int >= 1,
     "couplings": "ferromagnet" | {"pm_j_seed": int},
     "seed": int, "run_id": int, "capacity": int (0: the default),
     "theta": int >= 0, "scheme": "multinomial" | "poisson" | "nearest" | "systematic",
     "beta_f": float >= 0, "points": int >= 2}

The schedule is beta_i = i beta_f / (points - 1) (Sec. 2's steps between
beta_0 = 0 and beta_f; the points include both ends).  A file only names a
run: it changes no numerics.  The log line of step i holds beta_i, its
increment, ln Q_i (Eq. (1)), ln Z_hat_i (Eq. (7)), R_i, the moments, the
family statistics rho_t and S_f (Eq. (6)), the sampling variance of the
resampling (Eq. (5)) and, with ``timing``, the device time of its phases."""
import json

from . import pa, workloads

RUN_KEYS = {"workload", "dim", "L", "R", "couplings", "seed", "run_id", "capacity", "theta", "scheme",
            "beta_f", "points"}


def load_run(path):
    """The run description in ``path``, checked; raises ValueError."""
    with open(path) as fh:
        spec = json.load(fh)
    return check_run(spec)


def check_run(spec):
    missing, extra = RUN_KEYS - set(spec), set(spec) - RUN_KEYS
    if missing or extra:
        raise ValueError(f"run description: missing {sorted(missing)}, unknown {sorted(extra)}")
    if spec["dim"] not in (2, 3) or spec["L"] < 2 or spec["L"] % 2:
        raise ValueError("run description: dim must be 2 or 3 and L even and at least 2")
    if spec["R"] < 1 or spec["theta"] < 0 or spec["points"] < 2 or not spec["beta_f"] >= 0:
        raise ValueError("run description: R >= 1, theta >= 0, points >= 2, beta_f >= 0")
    if spec["scheme"] not in pa.SCHEMES:
        raise ValueError(f"run description: scheme must be one of {sorted(pa.SCHEMES)}")
    c = spec["couplings"]
    if not (c == "ferromagnet" or (isinstance(c, dict) and set(c) == {"pm_j_seed"})):
        raise ValueError('run description: couplings must be "ferromagnet" or {"pm_j_seed": seed}')
    return spec


def couplings_of(spec):
    c = spec["couplings"]
    return None if c == "ferromagnet" else workloads.pm_j_couplings(spec["dim"], spec["L"], c["pm_j_seed"])


def schedule_of(spec):
    return workloads.linear_schedule(spec["beta_f"], spec["points"])


def make_run(spec, stream=None):
    """A PARun at beta = 0 for the description."""
    return pa.PARun(spec["dim"], spec["L"], spec["R"], seed=spec["seed"], run_id=spec["run_id"],
                    capacity=spec["capacity"], couplings=couplings_of(spec), stream=stream)


def anneal(run, spec, log=None, timing=False):
    """The description's anneal on ``run`` (fresh, at beta = 0): per step
    reweight, resample, theta sweeps, observables, each step read back when
    it is done.  Returns the step records (step 0 is the initial sampling)
    and writes each as one JSON line to ``log`` (a writable text file) if
    given.  With ``timing`` the phases are bracketed by HIP events on the
    run's stream and each record gets their device times in ms."""
    import torch
    betas = schedule_of(spec)
    scheme, theta = spec["scheme"], spec["theta"]

    def mark():
        e = torch.cuda.Event(enable_timing=True)
        e.record(run.stream)
        return e

    rows = [_record(0, betas[0], 0.0, 0.0, run.free_energy(), run.observables())]
    _write(log, rows[0])
    for i in range(1, len(betas)):
        e = [mark()] if timing else []
        lnq = run.reweight(betas[i])
        run.resample(scheme)
        if timing:
            e.append(mark())
        run.sweep(theta)
        if timing:
            e.append(mark())
        ob = run.observables()
        rec = _record(i, betas[i], betas[i] - betas[i - 1], lnq, run.free_energy(), ob)
        if timing:
            e.append(mark())
            e[-1].synchronize()
            rec["ms"] = {"reweight_resample": e[0].elapsed_time(e[1]), "sweeps": e[1].elapsed_time(e[2]),
                         "observables": e[2].elapsed_time(e[3])}
        rows.append(rec)
        _write(log, rec)
    return rows


def _record(i, beta, dbeta, lnq, lnz, ob):
    keys = ("R", "e", "e2", "abs_m", "m2", "rho_t", "S_f", "sv", "families")
    rec = {"step": i, "beta": beta, "dbeta": dbeta, "lnQ": lnq, "lnZ": lnz}
    for k in keys:
        v = ob[k]
        rec[k] = int(v) if k in ("R", "families") else float(v)
    return rec


def _write(log, rec):
    if log is not None:
        log.write(json.dumps(rec) + "\n")
        log.flush()
