"""The surrogate network's HIP kernels against the FP64 reference (oracle/mlp.py)
with identical bfloat16-rounded weights."""
import sys

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device visible")
    from paper_1412_7228_amd import lbm as mod

    mod.load_library()
    return mod


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("n", [1, 31, 100, 1024])
def test_forward_matches_reference(lbm, n):
    say(f"mlp forward n={n}")
    net = lbm.MLP(max_batch=1024)
    p = omlp.init_params(11)
    net.set_params(p)
    x = np.random.default_rng(n).uniform(-1, 1, (n, 3)).astype(np.float32)
    y = net.forward(x)
    ref, _ = omlp.forward(p, x.astype(np.float64))
    assert _rel(y, ref) < 1e-5


@pytest.mark.parametrize("n", [7, 64, 333])
def test_backward_matches_reference(lbm, n):
    say(f"mlp backward n={n}")
    net = lbm.MLP(max_batch=512)
    p = omlp.init_params(12)
    net.set_params(p)
    g = np.random.default_rng(100 + n)
    x = g.uniform(-1, 1, (n, 3)).astype(np.float32)
    dy = g.normal(size=(n, 3)).astype(np.float32)
    grad, dx = net.backward(x, dy)
    rg, rdx = omlp.backward(p, x.astype(np.float64), dy.astype(np.float64))
    for w_off, shape, b_off, nb in omlp.LAYOUT:
        sl = slice(w_off, w_off + shape[0] * shape[1])
        assert _rel(grad[sl], rg[sl]) < 1e-4
        assert _rel(grad[b_off:b_off + nb], rg[b_off:b_off + nb]) < 1e-4
    assert _rel(dx, rdx) < 1e-4


def test_adam_step_matches_reference(lbm):
    say("mlp adam step")
    g = np.random.default_rng(3)
    x = g.uniform(-1, 1, (96, 3)).astype(np.float32)
    t = g.normal(size=(96, 3)).astype(np.float32)
    p = omlp.init_params(13)
    net = lbm.MLP(max_batch=128)
    net.set_params(p)
    net.set_data(x, t)
    loss = net.train(1, 1e-3)
    y, _ = omlp.forward(p, x.astype(np.float64))
    rl, dy = omlp.mse_loss_grad(y, t)
    assert abs(loss[0] / rl - 1) < 1e-5
    grad, _ = omlp.backward(p, x.astype(np.float64), dy)
    q, _, _ = omlp.adam_step(p.astype(np.float64), 0.0, 0.0, grad, 1, lr=1e-3)
    got = net.params()
    # the first Adam step moves each parameter by about lr * sign(g)
    assert np.abs(got - q).max() < 1e-6


def test_training_is_deterministic_and_learns(lbm):
    say("mlp training")
    g = np.random.default_rng(9)
    x = g.uniform(-1, 1, (200, 3)).astype(np.float32)
    t = np.stack([np.sin(2 * x[:, 0]) * x[:, 1], x[:, 2] ** 2 - 0.3, x[:, 0] - 0.5 * x[:, 1]], 1).astype(np.float32)
    runs = []
    for _ in range(2):
        net = lbm.MLP(max_batch=256)
        net.set_params(omlp.init_params(21))
        net.set_data(x, t)
        loss = net.train(400, 3e-3)
        runs.append((loss, net.params()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    loss = runs[0][0]
    assert loss[-1] < 0.05 * loss[0]


def test_forward_between_training_calls_leaves_training_set(lbm):
    """Forward and backward calls on other inputs between training calls (a
    held-out check) do not change what the next training call trains on."""
    say("mlp training interleaved with forward/backward")
    g = np.random.default_rng(11)
    x = g.uniform(-1, 1, (150, 3)).astype(np.float32)
    t = np.stack([x[:, 0] * x[:, 1], np.cos(x[:, 2]), x[:, 0] - x[:, 2]], 1).astype(np.float32)
    other = g.uniform(-1, 1, (200, 3)).astype(np.float32)
    runs = []
    for interleave in (False, True):
        net = lbm.MLP(max_batch=256)
        net.set_params(omlp.init_params(5))
        net.set_data(x, t)
        losses = []
        for _ in range(4):
            losses.append(net.train(25, 3e-3))
            if interleave:
                net.forward(other)
                net.backward(other, np.ones_like(other))
        runs.append((np.concatenate(losses), net.params()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


def test_surrogate_fit_and_inversion_on_a_smooth_law(lbm):
    """The surrogate pipeline (standardised targets, full-batch training with held-out
    selection, inversion for kappa on a dense grid) on a closed-form law of the shape
    Eq. (28) predicts, sigma = s0(A, T) (1 - kappa): the kappa it returns for a target
    reproduces the target within 2% of sigma (the tolerance of the tuning study)."""
    say("surrogate fit + inversion on a closed-form law")
    from paper_1412_7228_amd import surrogate as sg

    g = np.random.default_rng(4)
    n = 900
    A = g.uniform(-0.7, -0.3, n)
    k = g.uniform(0.0, 0.8, n)
    T = g.uniform(0.6, 0.85, n)

    def law(A, k, T):
        s0 = 0.05 * np.exp(-6.0 * (T - 0.6)) * (1.0 - 0.4 * A)
        return np.stack([s0 * (1.0 - k), 0.3 + 0.1 * A - 0.5 * (T - 0.6), 0.02 + 0.05 * (T - 0.6)], 1)

    X = np.stack([A, k, T], 1)
    sur = sg.Surrogate(seed=1, max_batch=1024)
    sur.fit(X, law(A, k, T), iters=4000, lr=1e-3, cosine=True)
    At = g.uniform(-0.65, -0.35, 20)
    Tt = g.uniform(0.62, 0.83, 20)
    kt = g.uniform(0.05, 0.75, 20)
    target = law(At, kt, Tt)[:, 0]
    kinv = sur.invert_kappa(At, Tt, target)
    got = law(At, kinv, Tt)[:, 0]
    assert np.abs(got / target - 1).max() < 0.02, np.abs(got / target - 1).max()
