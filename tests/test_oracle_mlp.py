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
