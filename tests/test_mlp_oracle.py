"""Pins of the surrogate oracle (CPU, FP64): every part checked against a
definition that does not reuse it."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M

SMALL = [5, 7, 6, 2]   # small widths for finite differences


def test_parameter_count():
    assert M.n_params() == 133634   # 5*256+256 + 2*(256*256+256) + 256*2+2


def test_gelu_and_its_derivative():
    x = np.linspace(-6, 6, 241)
    # GELU(x) = x Phi(x) with Phi the standard normal CDF (independent routine)
    from scipy.stats import norm
    assert np.allclose(M.gelu(x), x * norm.cdf(x), rtol=0, atol=1e-14)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.allclose(M.gelu_grad(x), fd, rtol=0, atol=1e-8)
    assert M.gelu(0.0) == 0.0 and abs(M.gelu_grad(0.0) - 0.5) < 1e-15


def test_round_bf16_against_bit_arithmetic():
    # 1 + 2^-8 is exactly between 1 and 1 + 2^-7: ties to even -> 1
    assert M.round_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert M.round_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6   # tie, odd neighbour below -> up
    assert M.round_bf16(np.array([1.0 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1.0 + 2.0 ** -7
    x = np.random.default_rng(0).normal(size=1000)
    r = M.round_bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * 1.0000001)
    assert np.all(M.round_bf16(r) == r)


@pytest.mark.parametrize("bf16", [False, True])
def test_gradient_matches_finite_differences(bf16):
    rng = np.random.default_rng(3)
    theta = M.init_params(1, SMALL) + rng.normal(scale=0.1, size=M.n_params(SMALL))
    X = rng.normal(size=(9, 5))
    T = rng.normal(size=(9, 2))
    Mk = (rng.random((9, 2)) > 0.3).astype(float)
    g = M.gradient(theta, X, T, Mk, bf16=False, layers=SMALL)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (M.loss(theta + e, X, T, Mk, False, SMALL) - M.loss(theta - e, X, T, Mk, False, SMALL)) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)
    if bf16:
        # with rounded operands the gradient is the FP64 gradient of the network
        # whose weights and layer inputs are those rounded values
        gb = M.gradient(theta, X, T, Mk, bf16=True, layers=SMALL)
        W = M.unpack(theta, SMALL)
        thr = np.concatenate([np.concatenate([M.round_bf16(w).ravel(), b]) for w, b in W])
        Xr = M.round_bf16(X)
        y_b, _ = M.forward(theta, X, True, SMALL)
        # the rounded network evaluated in FP64 on rounded inputs agrees for the first layer
        assert np.allclose(M.forward(thr, Xr, False, SMALL)[1][0][2], M.forward(theta, X, True, SMALL)[1][0][2])
        assert np.isfinite(gb).all() and np.abs(gb - g).max() < 5e-2 * np.abs(g).max()


def test_linear_case_closed_form():
    """One linear layer (no hidden GELU): loss = |XW + b - T|^2 / n, gradient
    2 X^T (XW + b - T) / n (least squares)."""
    layers = [5, 2]
    rng = np.random.default_rng(4)
    theta = rng.normal(size=M.n_params(layers))
    X, T = rng.normal(size=(11, 5)), rng.normal(size=(11, 2))
    Mk = np.ones((11, 2))
    W = theta[:10].reshape(5, 2)
    b = theta[10:]
    R = X @ W + b - T
    gW = 2 * X.T @ R / 22
    gb = 2 * R.sum(0) / 22
    g = M.gradient(theta, X, T, Mk, layers=layers)
    assert np.allclose(g[:10], gW.ravel(), atol=1e-13) and np.allclose(g[10:], gb, atol=1e-13)
    assert M.loss(theta, X, T, Mk, layers=layers) == pytest.approx(np.sum(R ** 2) / 22, rel=1e-14)


def test_adam_first_steps_by_hand():
    """Adam on f(x) = x^2 / 2 from x = 1 with lr = 0.1: the bias-corrected first
    step moves by lr * g / |g| = 0.1 exactly (up to eps)."""
    th, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    th1, m, v = M.adam_step(th, m, v, th.copy(), 1, 0.1)
    assert th1[0] == pytest.approx(0.9, abs=1e-9)
    assert m[0] == pytest.approx(0.1) and v[0] == pytest.approx(0.001)
    th2, m, v = M.adam_step(th1, m, v, th1.copy(), 2, 0.1)
    g2 = th1[0]   # 0.9 up to the eps of the first step
    m2 = 0.9 * 0.1 + 0.1 * g2
    v2 = 0.999 * 0.001 + 0.001 * g2 * g2
    step = 0.1 * (m2 / (1 - 0.81)) / (math.sqrt(v2 / (1 - 0.998001)) + 1e-8)
    assert th2[0] == pytest.approx(g2 - step, rel=1e-12)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(5)
    layers = [5, 32, 32, 2]
    theta = M.init_params(2, layers)
    X = rng.uniform(-1, 1, size=(256, 5))
    T = np.stack([np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2], X[:, 3] ** 2 - X[:, 4]], axis=1)
    Mk = np.ones_like(T)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    l0 = M.loss(theta, X, T, Mk, layers=layers)
    for t in range(1, 301):
        theta, m, v = M.adam_step(theta, m, v, M.gradient(theta, X, T, Mk, layers=layers), t, 3e-3)
    assert M.loss(theta, X, T, Mk, layers=layers) < 0.1 * l0
