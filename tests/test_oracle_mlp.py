"""Pins of the learned-step model's oracle: gradients by central finite
differences, Adam against its published update, bfloat16 rounding on known
values, features on closed-form populations (CPU only)."""
import math

import numpy as np

from oracle import mlp as Mo


def test_parameter_count_and_layout():
    assert Mo.NPARAMS == 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4801
    p = np.arange(Mo.NPARAMS, dtype=np.float64)
    d = Mo.unpack(p)
    assert d["W1"][0, 1] == 1 and d["b1"][0] == 512 and d["W2"][0, 0] == 576
    assert d["b3"][0] == 4800
    assert np.array_equal(Mo.pack(d), p)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = Mo.init_params(1).astype(np.float64) + 0.1 * rng.standard_normal(Mo.NPARAMS)
    X = rng.standard_normal((40, 8))
    y = rng.standard_normal(40)
    _, g = Mo.loss_and_grad(p, X, y)
    h = 1e-6
    for k in rng.choice(Mo.NPARAMS, 300, replace=False).tolist() + [0, 511, 4799, 4800]:
        e = np.zeros(Mo.NPARAMS)
        e[k] = h
        fd = (Mo.loss_and_grad(p + e, X, y)[0] - Mo.loss_and_grad(p - e, X, y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_adam_step():
    p, g = np.array([1.0, -2.0]), np.array([0.5, -0.25])
    m, v = np.zeros(2), np.zeros(2)
    p1, m1, v1 = Mo.adam(p, g, m, v, 1, 0.01)
    # first step: mh = g, vh = g^2, so the move is lr * sign(g) (up to eps)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-9)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_bf16_rounding():
    v = Mo.bf16(np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -3.0, 0.0],
                         np.float32))
    assert v.tolist() == [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -3.0, 0.0]


def test_features_closed_forms():
    f = Mo.features(np.full(100, -40), 16, 0.3, [], math.log(100))
    assert f.tolist() == [0.3, -2.5, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0]
    E = np.array([-8] * 50 + [8] * 50)
    f = Mo.features(E, 16, 0.1, [-0.5, -0.25], 0.0)
    assert abs(f[2] - 8 / 4) < 1e-15 and abs(f[3]) < 1e-15
    assert f[4] == 0.0 and f[5] == -0.5 / 16 and f[6] == -0.25 / 16 and f[7] == 0.0
    # exponential-like energies are skewed to the right
    Ex = np.random.default_rng(1).exponential(10, 20000)
    assert abs(Mo.features(Ex, 1, 0, [], 0)[3] - 2.0) < 0.2


def test_training_fits_a_smooth_target():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((256, 8))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1]
    p = Mo.init_params(3).astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    l0 = Mo.loss_and_grad(p, X, y)[0]
    for t in range(1, 301):
        loss, g = Mo.loss_and_grad(p, X, y)
        p, m, v = Mo.adam(p, g, m, v, t, 1e-2)
    assert loss < 0.05 * l0
    # bfloat16 inference stays close to float64
    assert np.max(np.abs(Mo.forward_bf16(p, X) - Mo.forward(p, X)[0])) < 0.1
