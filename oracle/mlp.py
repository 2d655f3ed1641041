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


# --------------------------------------------------------------------------------------------
# BF16 inference: the network with BF16 weights, and a bound on what the rest of the rounding adds
# --------------------------------------------------------------------------------------------
BF16_UNIT = 2.0 ** -8        # unit roundoff of bfloat16 (8 significant bits), round to nearest even
FP32_UNIT = 2.0 ** -24


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), via FP32; returned as float64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _gamma(n):
    return n * FP32_UNIT / (1.0 - n * FP32_UNIT)


def bf16_inference(theta, x):
    """Standardised heads of the network whose weight matrices are rounded to BF16 (biases kept as
    given), evaluated in FP64, and a first-order bound per point and head on how far an evaluation
    that also (i) rounds the features to FP32, (ii) accumulates every layer's products in FP32,
    (iii) evaluates SiLU in FP32 and (iv) rounds every hidden activation to BF16 can lie from it.

    The bound is a running error bound carried forward through the layers: an error e in a layer's
    inputs reaches its pre-activations as |W| e; FP32 accumulation of n products adds at most
    gamma_n (|W| |h| + |b|), gamma_n = n u / (1 - n u); SiLU passes an error through with |SiLU'|
    and adds its own evaluation error, bounded by (8 + 2|a|) u |SiLU(a)|; rounding to BF16 adds
    BF16_UNIT |h|.  Second-order terms are neglected (each is below 1e-3 of the first-order ones).
    """
    p = unpack(theta)
    W = {k: bf16_round(p[k]) for k in ("W1", "W2", "W3", "W4")}
    x = np.asarray(x, np.float64)
    e = FP32_UNIT * np.abs(x)                       # features rounded to FP32
    h = x
    for k, b in (("W1", "b1"), ("W2", "b2"), ("W3", "b3")):
        a = h @ W[k].T + p[b]
        n = W[k].shape[1] + 1
        ea = e @ np.abs(W[k]).T + _gamma(n) * (np.abs(h) @ np.abs(W[k]).T + np.abs(p[b]))
        hn = silu(a)
        e = np.abs(dsilu(a)) * ea + (8.0 + 2.0 * np.abs(a)) * FP32_UNIT * np.abs(hn) + BF16_UNIT * np.abs(hn)
        h = hn
    y = h @ W["W4"].T + p["b4"]
    ey = e @ np.abs(W["W4"]).T + _gamma(W["W4"].shape[1] + 1) * (np.abs(h) @ np.abs(W["W4"]).T + np.abs(p["b4"]))
    return y, ey + FP32_UNIT * np.abs(y)
