"""Host side of the run descriptions (paper_2401_07965_amd/runs/*.json):
every shipped file passes the checks and names the schedule, couplings and
sizes it says; malformed descriptions are rejected."""
import glob
import json
import os

import numpy as np
import pytest

from paper_2401_07965_amd import driver, workloads

RUNS = sorted(glob.glob(os.path.join(os.path.dirname(driver.__file__), "runs", "*.json")))


def test_shipped_runs_load():
    assert len(RUNS) == 8
    for path in RUNS:
        spec = driver.load_run(path)
        betas = driver.schedule_of(spec)
        assert len(betas) == spec["points"] and betas[0] == 0.0 and betas[-1] == spec["beta_f"]
        assert all(b1 > b0 for b0, b1 in zip(betas, betas[1:]))
        J = driver.couplings_of(spec)
        if spec["couplings"] == "ferromagnet":
            assert J is None
        else:
            assert J.shape == (spec["L"] ** spec["dim"] * spec["dim"],) and set(np.unique(J)) <= {-1, 1}


def test_glass_populations_share_their_couplings():
    a = driver.load_run(os.path.join(os.path.dirname(driver.__file__), "runs", "3d_pmj_L10_R5e5_A.json"))
    b = driver.load_run(os.path.join(os.path.dirname(driver.__file__), "runs", "3d_pmj_L10_R5e5_B.json"))
    assert np.array_equal(driver.couplings_of(a), driver.couplings_of(b))
    assert a["run_id"] != b["run_id"]
    assert np.array_equal(driver.couplings_of(a), workloads.pm_j_couplings(3, 10, 1))


@pytest.mark.parametrize("change", [{"dim": 4}, {"L": 7}, {"R": 0}, {"points": 1}, {"scheme": "stratified"},
                                    {"couplings": "glass"}, {"beta_f": -1.0}, {"extra": 1}])
def test_malformed_runs_are_rejected(change, tmp_path):
    spec = driver.load_run(RUNS[0])
    spec.update(change)
    p = tmp_path / "bad.json"
    p.write_text(json.dumps(spec))
    with pytest.raises(ValueError):
        driver.load_run(str(p))


def test_missing_key_is_rejected():
    spec = driver.load_run(RUNS[0])
    del spec["theta"]
    with pytest.raises(ValueError):
        driver.check_run(spec)
