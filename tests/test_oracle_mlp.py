"""Pins of the surrogate network's FP64 reference (oracle/mlp.py)."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_parameter_count():
    # 3->128->128->128->3 with biases
    assert mlp.NPARAMS == 3 * 128 + 128 + 128 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3 == 33923


def test_bf16_rounding_matches_torch():
    g = np.random.default_rng(0)
    x = np.concatenate([g.normal(size=20000).astype(np.float32),
                        np.array([1.0, -2.5, 3.00390625, 1.00390625, 1.01171875], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_gradients_match_finite_differences():
    g = np.random.default_rng(1)
    p = mlp.init_params(3).astype(np.float64)
    x = g.uniform(-1, 1, (5, 3))
    dy = g.normal(size=(5, 3))
    grad, dx = mlp.backward(p, x, dy, round_weights=False)
    f = lambda q, xx: float(np.sum(dy * mlp.forward(q, xx, round_weights=False)[0]))
    idx = g.choice(mlp.NPARAMS, 60, replace=False)
    for i in list(idx) + [0, mlp.NPARAMS - 1, mlp.LAYOUT[2][0] + 5]:
        h = 1e-6
        e = np.zeros_like(p)
        e[i] = h
        fd = (f(p + e, x) - f(p - e, x)) / (2 * h)
        assert abs(fd - grad[i]) < 1e-7 * max(1.0, abs(fd)), i
    for r in range(5):
        for k in range(3):
            e = np.zeros_like(x)
            e[r, k] = 1e-6
            fd = (f(p, x + e) - f(p, x - e)) / 2e-6
            assert abs(fd - dx[r, k]) < 1e-7 * max(1.0, abs(fd))


def test_rounded_weights_are_what_the_gradient_sees():
    p = mlp.init_params(4)
    x = np.random.default_rng(2).uniform(-1, 1, (7, 3))
    y1, _ = mlp.forward(p, x)
    q = p.astype(np.float64).copy()
    for w_off, shape, _, _ in mlp.LAYOUT:
        n = shape[0] * shape[1]
        q[w_off:w_off + n] = mlp.bf16_round(p[w_off:w_off + n])
    y2, _ = mlp.forward(q, x, round_weights=False)
    assert np.array_equal(y1, y2)


def test_adam_first_step_moves_by_lr():
    p = np.zeros(10)
    grad = np.linspace(-1, 1, 10)
    grad[5] = 0.3
    q, m, v = mlp.adam_step(p, np.zeros(10), np.zeros(10), grad, 1, lr=0.01)
    # bias-corrected first step is lr * sign(g) (up to eps)
    assert np.allclose(q, -0.01 * np.sign(grad), atol=1e-9)


def test_training_reduces_loss_on_a_smooth_target():
    g = np.random.default_rng(5)
    x = g.uniform(-1, 1, (64, 3))
    t = np.stack([np.sin(x[:, 0]) * x[:, 1], x[:, 2] ** 2, x[:, 0] - x[:, 1]], axis=1)
    p = mlp.init_params(7).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for it in range(1, 201):
        y, _ = mlp.forward(p, x, round_weights=False)
        loss, dy = mlp.mse_loss_grad(y, t)
        grad, _ = mlp.backward(p, x, dy, round_weights=False)
        p, m, v = mlp.adam_step(p, m, v, grad, it, lr=3e-3)
        losses.append(loss)
    assert losses[-1] < 0.05 * losses[0]
