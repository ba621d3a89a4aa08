"""CPU checks of the adaptive-anneal driver's sequencing (no GPU): it follows
the steps the rule returns, and it stops with an error instead of looping
when the rule returns no step that moves beta."""
import pytest

from paper_2401_07965_amd.schedule import NoStepError, anneal_adaptive


class FakeRun:
    """Stands in for pa.PARun: returns scripted steps and records the calls."""

    def __init__(self, steps):
        self.steps = list(steps)
        self.betas = []

    def observables(self, wait=True):
        return {}

    def step_rule(self, alpha_star, dbeta_max, iterations=60):
        return self.steps.pop(0) if self.steps else dbeta_max

    def step_learned(self, mlp, alpha_star, dbeta_max, iterations=60, bracket=1.0, refine=0):
        return self.step_rule(alpha_star, dbeta_max, iterations), False

    def reweight(self, beta, wait=True):
        self.betas.append(beta)

    def resample(self, scheme, wait=True):
        return 1

    def sweep(self, theta):
        pass

    def free_energy(self):
        return 0.0


def test_follows_the_rule_and_ends_at_beta_f():
    run = FakeRun([0.25, 0.5, 0.25])
    out = anneal_adaptive(run, 1.0, 0.7, 0.5, 1, 3)
    assert run.betas == [0.25, 0.75, 1.0]
    assert out["steps"] == 3 and out["betas"] == [0.0, 0.25, 0.75, 1.0]


@pytest.mark.parametrize("d", [0.0, -1.0, 1e-30])
def test_no_moving_step_raises(d):
    # 1e-30 is below half an ulp of beta = 0.25: beta + d == beta
    run = FakeRun([0.25, d])
    with pytest.raises(NoStepError):
        anneal_adaptive(run, 1.0, 0.7, 0.5, 1, 3)
    assert run.betas == [0.25]


def test_step_cap():
    run = FakeRun([1e-3] * 50)
    with pytest.raises(NoStepError):
        anneal_adaptive(run, 1.0, 0.7, 0.5, 1, 3, max_steps=10)
    assert len(run.betas) == 10


def test_learned_and_deferred_paths_sequence_the_same_calls():
    run = FakeRun([0.5, 0.5])
    out = anneal_adaptive(run, 1.0, 0.7, 0.5, 1, 3, mlp=object(), bracket=1.25, refine=6, deferred=True)
    assert run.betas == [0.5, 1.0] and out["fallbacks"] == 0 and out["steps"] == 2
