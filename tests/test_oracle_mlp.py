"""The oracle's functional surrogate (FP64 MLP) against calculus and the Adam definition (no GPU)."""
import math

import numpy as np

from oracle import functionals as fx
from oracle import mlp


def test_parameter_count_and_layout():
    assert mlp.N_PARAMS == 8707
    rng = np.random.default_rng(0)
    th = mlp.init_params(rng)
    p = mlp.unpack(th)
    assert p["W2"].shape == (64, 64) and p["W4"].shape == (3, 64) and p["b4"].shape == (3,)
    assert np.array_equal(mlp.pack(p), th)
    assert np.all(p["b1"] == 0) and np.abs(p["W1"]).max() <= 1 / math.sqrt(2)


def test_backprop_matches_central_differences():
    rng = np.random.default_rng(1)
    th = mlp.init_params(rng) + 0.05 * rng.normal(size=mlp.N_PARAMS)
    x = rng.uniform(-1, 1, size=(17, 2))
    s = rng.normal(size=(17, 3))
    L, g = mlp.loss_and_grad(th, x, s)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(th + e, x, s)[0] - mlp.loss_and_grad(th - e, x, s)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * abs(g[i]) + 5e-10   # rounding floor of the quotient ~ eps L / h


def test_silu_derivative():
    a = np.linspace(-8, 8, 101)
    h = 1e-6
    assert np.allclose(mlp.dsilu(a), (mlp.silu(a + h) - mlp.silu(a - h)) / (2 * h), atol=1e-9)


def test_adam_first_step_is_signed_lr():
    # with zero moments, the bias-corrected first step is lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_features_and_targets_round_trip():
    box = (math.log(1e-8), math.log(10.0), math.log(1e-30), math.log(1e3))
    x = mlp.features(np.array([1e-8, 10.0]), np.array([0.0, 1e3]), box)
    assert np.allclose(x, [[-1, -1], [1, 1]])
    rho = np.array([1e-3, 0.5, 7.0])
    sig = np.array([1e-6, 0.2, 30.0])
    f, vr, vs = fx.evaluate("pbe", rho, sig, 0.0)
    t = mlp.targets(rho, f, vr, vs)
    f2, vr2, vs2 = mlp.from_targets(rho, t)
    assert np.allclose(f2, f, rtol=1e-14) and np.allclose(vr2, vr, rtol=1e-14) and np.allclose(vs2, vs, rtol=1e-14)
    # exchange-like heads are O(1): f_x / rho^{4/3} = -C_x F_x in [-1.804 C_x, -C_x]
    fxx, _, _ = fx.pbe_x(rho, sig)
    assert np.all(np.abs(fxx / rho ** (4 / 3)) <= 1.804 * fx.CX + 1e-12)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(2)
    th = mlp.init_params(rng)
    x = rng.uniform(-1, 1, size=(256, 2))
    s = np.stack([np.sin(2 * x[:, 0]), x[:, 1] ** 2 - 0.3, x[:, 0] * x[:, 1]], axis=1)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0 = mlp.loss_and_grad(th, x, s)[0]
    for k in range(1, 301):
        L, g = mlp.loss_and_grad(th, x, s)
        th, m, v = mlp.adam_step(th, g, m, v, k, lr=3e-3)
    assert mlp.loss_and_grad(th, x, s)[0] < 0.1 * L0


def test_bf16_round_known_values():
    # 8 significant bits: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 and ties to the even 1;
    # 1 + 3*2^-8 ties to the even 1 + 2^-6; 1 + 2^-8 + 2^-20 rounds up
    v = mlp.bf16_round(np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, -3.0, 0.0]))
    assert np.array_equal(v, [1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -3.0, 0.0])
    r = np.random.default_rng(0).normal(size=10000) * 10.0 ** np.random.default_rng(1).uniform(-5, 5, 10000)
    q = mlp.bf16_round(r)
    assert np.all(np.abs(q - r) <= mlp.BF16_UNIT * np.abs(r) * (1 + 1e-6))
    assert np.array_equal(mlp.bf16_round(q), q)


def test_bf16_inference_bound_holds_for_an_emulation():
    """Brute force: the network evaluated in numpy float32 with BF16 weights and every hidden
    activation rounded to BF16 lies within the bound of bf16_inference, and the bound is not vacuous
    (the largest emulated error is a visible share of it: rounding errors of a 64-term sum mostly
    cancel, which the worst-case bound does not assume)."""
    rng = np.random.default_rng(2)
    th = mlp.init_params(rng) + 0.1 * rng.normal(size=mlp.N_PARAMS)
    x = rng.uniform(-1, 1, size=(3000, 2))
    y, ey = mlp.bf16_inference(th, x)
    p = mlp.unpack(th)
    W = {k: mlp.bf16_round(p[k]).astype(np.float32) for k in ("W1", "W2", "W3", "W4")}
    h = x.astype(np.float32)
    for k, b in (("W1", "b1"), ("W2", "b2"), ("W3", "b3")):
        a = (h @ W[k].T + p[b].astype(np.float32)).astype(np.float32)
        h = mlp.bf16_round(a / (np.float32(1) + np.exp(-a))).astype(np.float32)
    ye = (h @ W["W4"].T + p["b4"].astype(np.float32)).astype(np.float64)
    d = np.abs(ye - y)
    assert np.all(d <= ey)
    assert (d / ey).max() > 0.01
    # the BF16 weights alone move the heads by far more than the bound's FP32 terms
    y64, _ = mlp.forward(th, x)
    assert np.abs(y64 - y).max() > 10 * mlp.FP32_UNIT * np.abs(y).max()
