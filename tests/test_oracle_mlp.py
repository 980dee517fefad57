"""Pins of the FP64 screener-network reference: central finite differences of the
loss, the loss of a zero network, and the Adam update against its closed form."""
import numpy as np

import gen
from oracle import mlp


def _batch(seed=1, B=6):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, 32)), (rng.uniform(size=(B, 4)) > 0.5).astype(float)


def test_param_count_and_layout():
    th = gen.mlp_init(7)
    assert th.size == gen.mlp_param_count() == 21252
    layers = mlp.unpack(th)
    assert [W.shape for W, _ in layers] == [(32, 128), (128, 128), (128, 4)]
    assert np.all(np.abs(layers[0][0]) <= 1 / np.sqrt(32) + 1e-7)


def test_zero_network_loss_is_log2():
    X, Y = _batch()
    assert abs(mlp.loss(np.zeros(21252), X, Y) - np.log(2.0)) < 1e-15


def test_gradient_matches_central_differences():
    X, Y = _batch(3, 5)
    th = gen.mlp_init(7).astype(np.float64)
    L, g = mlp.loss_and_grad(th, X, Y)
    rng = np.random.default_rng(0)
    # parameters from every layer, weights and biases
    idx = np.concatenate([rng.choice(4096, 6, replace=False), 4096 + rng.choice(128, 3, replace=False),
                          4224 + rng.choice(16384, 6, replace=False), 20608 + rng.choice(128, 3, replace=False),
                          20736 + rng.choice(512, 6, replace=False), 21248 + np.arange(4)])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        fd = (mlp.loss(th + e, X, Y) - mlp.loss(th - e, X, Y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-8 + 1e-6 * abs(fd), (k, fd, g[k])


def test_output_bias_gradient_is_mean_residual():
    X, Y = _batch(4, 7)
    th = gen.mlp_init(7).astype(np.float64)
    _, _, p = mlp.forward(th, X)
    _, g = mlp.loss_and_grad(th, X, Y)
    assert np.allclose(g[-4:], (p - Y).sum(axis=0) / (7 * 4), atol=1e-15)


def test_adam_first_step_moves_by_lr():
    th = np.ones(5)
    g = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    new, m, v = mlp.adam_step(th, g, np.zeros(5), np.zeros(5), 1, lr=1e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> step = lr * sign(g) (g != 0)
    expect = th - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(new, expect, rtol=0, atol=1e-15)
