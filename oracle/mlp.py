"""Learned functional surrogate -- oracle, FP64 (test infrastructure only).

A small multilayer perceptron stands in for the GGA functional evaluation (the learned form of the
workload; not in the paper):

    input   x = (n(log rho), n(log sigma)),  n(.) an affine map of the training range box onto
            [-1, 1], sigma floored at 1e-30 before the log;
    hidden  h1 = SiLU(W1 x + b1), h2 = SiLU(W2 h1 + b2), h3 = SiLU(W3 h2 + b3), width 64,
            SiLU(a) = a / (1 + exp(-a));
    output  y = W4 h3 + b4 (3 heads), de-standardised t = y * t_std + t_mean;
    heads   t0 = f / rho^{4/3},  t1 = v_rho / rho^{1/3},  t2 = v_sigma * rho^{4/3}  (dimensionless,
            O(1) for exchange-like forms), so f = t0 rho^{4/3}, v_rho = t1 rho^{1/3},
            v_sigma = t2 / rho^{4/3}.

Loss of a batch: L = (1 / (3B)) sum_{points, heads} (y - s)^2 with standardised targets
s = (t - t_mean) / t_std.  Parameters are updated by Adam (Kingma & Ba 2015):
    m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
    theta -= lr * (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps).

The three heads are independent, so the surrogate's v_rho, v_sigma are not exact derivatives of its
f (the analytic functional's are).
"""
from __future__ import annotations

import math

import numpy as np

WIDTH = 64
SIGMA_FLOOR = 1e-30
SHAPES = [("W1", (WIDTH, 2)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (3, WIDTH)), ("b4", (3,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)     # 8707


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], np.float64).ravel() for name, _ in SHAPES])


def silu(a):
    return a / (1.0 + np.exp(-a))


def dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def features(rho, sigma, box):
    """box = (lr_min, lr_max, ls_min, ls_max) of log rho and log sigma."""
    lr = np.log(rho)
    ls = np.log(np.maximum(sigma, SIGMA_FLOOR))
    x0 = 2.0 * (lr - box[0]) / (box[1] - box[0]) - 1.0
    x1 = 2.0 * (ls - box[2]) / (box[3] - box[2]) - 1.0
    return np.stack([x0, x1], axis=1)


def forward(theta, x):
    """Standardised outputs y (B x 3) and the pre-activations kept for the backward pass."""
    p = unpack(theta)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = silu(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(a2)
    a3 = h2 @ p["W3"].T + p["b3"]
    h3 = silu(a3)
    y = h3 @ p["W4"].T + p["b4"]
    return y, (x, a1, h1, a2, h2, a3, h3)


def loss_and_grad(theta, x, s):
    """L = mean over points and heads of (y - s)^2, and dL/dtheta (back-propagation)."""
    p = unpack(theta)
    y, (x, a1, h1, a2, h2, a3, h3) = forward(theta, x)
    B = x.shape[0]
    r = y - s
    L = float(np.sum(r * r) / (3.0 * B))
    gy = 2.0 * r / (3.0 * B)
    g = {}
    g["W4"] = gy.T @ h3
    g["b4"] = gy.sum(0)
    d3 = (gy @ p["W4"]) * dsilu(a3)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(0)
    d2 = (d3 @ p["W3"]) * dsilu(a2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * dsilu(a1)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(0)
    return L, pack(g)


def init_params(rng):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    params = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = 1.0 / math.sqrt(shp[1])
            params[name] = rng.uniform(-lim, lim, size=shp)
        else:
            params[name] = np.zeros(shp)
    return pack(params)


def adam_step(theta, g, m, v, k, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** k)
    vh = v / (1.0 - b2 ** k)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def targets(rho, f, vr, vs):
    r13 = np.cbrt(rho)
    r43 = rho * r13
    return np.stack([f / r43, vr / r13, vs * r43], axis=1)


def from_targets(rho, t):
    r13 = np.cbrt(rho)
    r43 = rho * r13
    return t[:, 0] * r43, t[:, 1] * r13, t[:, 2] / r43
