"""The run-description driver on the GPU: the 2D L = 8, R = 1000 description
annealed with a per-step JSON log (and device timings) agrees with the oracle
at every step (ln Q within 1e-10, R and ln Z_hat), and the log holds one
parseable line per step with the documented fields."""
import io
import json
import os

import pytest

from oracle import oracle as O
from paper_2401_07965_amd import driver
from tests.paritylib import rel_ok

pytestmark = pytest.mark.gpu


def test_logged_anneal_matches_the_oracle():
    spec = driver.load_run(os.path.join(os.path.dirname(driver.__file__), "runs", "2d_fm_L8_R1000_nearest.json"))
    run = driver.make_run(spec)
    log = io.StringIO()
    rows = driver.anneal(run, spec, log=log, timing=True)
    run.close()
    betas = driver.schedule_of(spec)
    assert len(rows) == len(betas)
    o = O.OracleRun(spec["dim"], spec["L"], spec["R"], seed=spec["seed"], run_id=spec["run_id"])
    for i, b in enumerate(betas[1:], 1):
        q = o.reweight(b)
        R = o.resample(O.NEAREST_INT)
        o.sweep(spec["theta"])
        assert rel_ok(rows[i]["lnQ"], q), (i, rows[i]["lnQ"], q)
        assert rows[i]["R"] == R, i
        assert rel_ok(rows[i]["lnZ"], o.lnZ), i
    lines = [json.loads(x) for x in log.getvalue().splitlines()]
    assert [x["step"] for x in lines] == list(range(len(betas)))
    for x in lines[1:]:
        assert set(x) >= {"beta", "dbeta", "lnQ", "lnZ", "R", "e", "e2", "abs_m", "m2", "rho_t", "S_f", "sv",
                          "families", "ms"}
        assert all(v >= 0.0 for v in x["ms"].values())
