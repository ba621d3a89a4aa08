"""GPU tests of the learned temperature-step model: gradients and Adam steps
of the float32 training kernels against the float64 oracle, bfloat16
inference against the oracle's bfloat16 emulation, the model inputs of a
population, and the exact check of a proposal."""
import math

import numpy as np
import pytest

from oracle import mlp as Mo
from oracle import oracle as O
from oracle import schedule as S
from tests.paritylib import rel_ok, run_pair, schedule

pytestmark = pytest.mark.gpu


def data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 8)).astype(np.float32) * np.arange(1, 9, dtype=np.float32)
    y = (np.sin(X[:, 0]) + 0.1 * X[:, 1] - 3.0).astype(np.float32)
    xm, xs = X.mean(axis=0), X.std(axis=0)
    return X, y, xm, xs, float(y.mean()), float(y.std())


def normalised(X, y, xm, xs, ym, ys):
    Xn = ((X - xm) / xs).astype(np.float32).astype(np.float64)
    yn = float(np.float32(1.0)) * ((y - np.float32(ym)) / np.float32(ys)).astype(np.float64)
    return Xn, yn


def test_gradient_matches_oracle():
    from paper_2401_07965_amd import pa
    X, y, xm, xs, ym, ys = data(300, 0)
    p = Mo.init_params(4)
    m = pa.PAMlp(p, xm, xs, ym, ys, max_samples=512)
    m.set_data(X, y)
    g, loss = m.gradient()
    Xn, yn = normalised(X, y, xm, xs, ym, ys)
    lo, go = Mo.loss_and_grad(p.astype(np.float64), Xn, yn)
    assert abs(loss - lo) <= 1e-5 * lo
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    assert np.all(np.abs(g[big] - go[big]) <= 1e-3 * np.abs(go[big]) + 1e-6)
    m.close()


def test_adam_training_tracks_oracle():
    from paper_2401_07965_amd import pa
    X, y, xm, xs, ym, ys = data(256, 1)
    p = Mo.init_params(5)
    m = pa.PAMlp(p, xm, xs, ym, ys, max_samples=256)
    m.set_data(X, y)
    m.train(20, 1e-2)
    Xn, yn = normalised(X, y, xm, xs, ym, ys)
    po, mo, vo = p.astype(np.float64), np.zeros(Mo.NPARAMS), np.zeros(Mo.NPARAMS)
    for t in range(1, 21):
        _, go = Mo.loss_and_grad(po, Xn, yn)
        po, mo, vo = Mo.adam(po, go, mo, vo, t, 1e-2)
    pg = m.params()
    assert np.max(np.abs(pg - po)) < 2e-3
    l_end = m.train(200, 1e-2)
    assert l_end < 0.2 * Mo.loss_and_grad(p.astype(np.float64), Xn, yn)[0]
    m.close()


def test_bf16_inference_matches_emulation():
    from paper_2401_07965_amd import pa
    X, y, xm, xs, ym, ys = data(200, 2)
    p = Mo.init_params(6)
    m = pa.PAMlp(p, xm, xs, ym, ys, max_samples=256)
    m.set_data(X, y)
    m.train(100, 1e-2)
    pt = m.params()
    got = m.predict(X)
    Xn = ((X - xm) / xs).astype(np.float32)
    yb = Mo.forward_bf16(pt.astype(np.float64), Xn)
    ref = np.exp(yb.astype(np.float64) * ys + ym)
    assert np.max(np.abs(got / ref - 1)) < 0.02
    y32 = Mo.forward(pt.astype(np.float64), Xn.astype(np.float64))[0]
    assert np.max(np.abs(got / np.exp(y32 * ys + ym) - 1)) < 0.1
    m.close()


def test_features_and_learned_check():
    from paper_2401_07965_amd import pa
    betas = schedule(0.6, 7)
    g, o = run_pair(2, 8, 1000, O.NEAREST_INT, betas, 4, observables=True)
    f = g.features()
    ob = o.observables()
    lnq = [o.reweight(b) for b in ()]  # no extra step
    st = g.export()
    hist = []
    oo = O.OracleRun(2, 8, 1000, seed=1, run_id=0)
    for b in betas[1:]:
        hist.append(oo.reweight(b))
        oo.resample(O.NEAREST_INT)
        oo.sweep(4)
    ref = Mo.features(st["energy"], 64, betas[-1], hist, ob["S_f"])
    assert np.allclose(f, ref.astype(np.float32), rtol=1e-6, atol=1e-7), (f, ref)
    # a model whose proposal is too large falls back to the exact rule
    X = np.tile(f, (8, 1))
    p = np.zeros(Mo.NPARAMS, np.float32)
    for logd, expect_fallback in ((math.log(0.5), True), (math.log(1e-4), False)):
        m = pa.PAMlp(p, np.zeros(8), np.ones(8), logd, 1.0, max_samples=8)
        d, fb = g.step_learned(m, 0.8, 0.5, 60)
        assert fb == expect_fallback
        if fb:
            assert d == S.step_rule(st["energy"], 0.8, 0.5, 60)
        else:
            assert d == float(np.exp(np.float32(0.0) * 1.0 + logd)) or rel_ok(d, 1e-4, 1e-6)
            assert S.qualifies(st["energy"], d, S.target(0.8))
        m.close()
    # proposals refined in a bracket: exactly the oracle's steps, fallbacks included
    rule = S.step_rule(st["energy"], 0.8, 0.5, 60)
    for f in (0.02, 0.5, 0.9, 0.99, 1.0, 1.01, 1.1, 1.3, 5.0):
        m = pa.PAMlp(p, np.zeros(8), np.ones(8), math.log(f * rule), 1.0, max_samples=8)
        for bracket, refine in ((1.25, 6), (2.0, 10), (1.0, 0)):
            d, fb, c = g.step_learned(m, 0.8, 0.5, 60, bracket, refine, proposal=True)
            ref, rfb = S.learned_step(st["energy"], c, 0.8, 0.5, 60, bracket, refine)
            assert (d, fb) == (ref, rfb), (f, bracket, refine, d, ref)
        m.close()
    g.close()
