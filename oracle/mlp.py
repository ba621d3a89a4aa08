"""Oracle of the learned temperature-step model (test infrastructure only).

Not part of the paper: a small network proposes the next inverse-temperature
step from population statistics; the exact overlap rule (oracle/schedule.py)
stays as its arbiter and fallback.  This module is the plain float64 version
of everything the GPU computes for it, pinned by finite differences:

* features of a population (8 numbers): beta, <E>/N, sd(E)/sqrt(N),
  skewness of E, the last three ln Q divided by N (Eq. (1); 0 before they
  exist) and the family entropy over ln R;
* the network 8 -> 64 -> 64 -> 1 with tanh hidden layers on standardised
  inputs, predicting the standardised ln(dbeta); parameters in one flat
  vector: W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3;
* loss (1/2n) sum (y_hat - y)^2, its gradient, and Adam (Kingma & Ba 2015);
* bfloat16 inference: weights and each layer's inputs rounded to bfloat16
  (nearest, ties to even), sums in float32.
"""
import math

import numpy as np

H = 64
SIZES = dict(W1=(H, 8), b1=(H,), W2=(H, H), b2=(H,), W3=(H,), b3=(1,))
NPARAMS = sum(int(np.prod(s)) for s in SIZES.values())  # 4801


def unpack(p):
    out, k = {}, 0
    for name, shape in SIZES.items():
        n = int(np.prod(shape))
        out[name] = np.asarray(p[k:k + n], np.float64).reshape(shape)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[n], np.float64).reshape(-1) for n in SIZES])


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SIZES.items():
        if name.startswith("W"):
            fan_in = shape[-1] if len(shape) == 2 else H
            d[name] = rng.uniform(-1, 1, shape) / math.sqrt(fan_in)
        else:
            d[name] = np.zeros(shape)
    return pack(d).astype(np.float32)


def features(E, N, beta, lnq_hist, S_f):
    """Eight inputs of the model for a population with energies E."""
    E = np.asarray(E, np.float64)
    R = len(E)
    mean = E.mean()
    var = ((E - mean) ** 2).mean()
    m3 = ((E - mean) ** 3).mean()
    skew = m3 / var ** 1.5 if var > 0 else 0.0
    q = list(lnq_hist)[-3:]
    q = [0.0] * (3 - len(q)) + q
    return np.array([beta, mean / N, math.sqrt(var) / math.sqrt(N), skew,
                     q[0] / N, q[1] / N, q[2] / N, S_f / math.log(R) if R > 1 else 0.0])


def forward(p, Xn):
    d = unpack(p)
    Z1 = Xn @ d["W1"].T + d["b1"]
    H1 = np.tanh(Z1)
    Z2 = H1 @ d["W2"].T + d["b2"]
    H2 = np.tanh(Z2)
    y = H2 @ d["W3"] + d["b3"][0]
    return y, (H1, H2)


def loss_and_grad(p, Xn, yn):
    n = len(yn)
    d = unpack(p)
    yh, (H1, H2) = forward(p, Xn)
    r = yh - yn
    loss = 0.5 * float(r @ r) / n
    dY = r / n
    g = {"W3": H2.T @ dY, "b3": np.array([dY.sum()])}
    D2 = np.outer(dY, d["W3"]) * (1 - H2 ** 2)
    g["W2"] = D2.T @ H1
    g["b2"] = D2.sum(axis=0)
    D1 = (D2 @ d["W2"]) * (1 - H1 ** 2)
    g["W1"] = D1.T @ Xn
    g["b1"] = D1.sum(axis=0)
    return loss, pack(g)


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16(x):
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    a = np.asarray(x, np.float32).copy()
    u = a.view(np.uint32)
    u += np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    u &= np.uint32(0xFFFF0000)
    return a


def forward_bf16(p, Xn):
    """bfloat16 weights and layer inputs, float32 sums."""
    d = {k: bf16(v.astype(np.float32)) for k, v in unpack(p).items()}
    x = bf16(np.asarray(Xn, np.float32))
    h1 = bf16(np.tanh((x @ d["W1"].T + d["b1"]).astype(np.float32)))
    h2 = bf16(np.tanh((h1 @ d["W2"].T + d["b2"]).astype(np.float32)))
    return (h2 @ d["W3"] + d["b3"][0]).astype(np.float32)
