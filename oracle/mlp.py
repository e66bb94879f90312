"""FP64 reference of the surrogate network's forward, backward and Adam step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The surrogate maps (A, kappa, T/Tc), normalised, to (sigma, rho_l, rho_v),
normalised: 3 -> 128 -> 128 -> 128 -> 3, tanh on the hidden layers, a linear
output layer.  The weights are used rounded to bfloat16 (round to nearest,
ties to even); biases, activations and every sum are FP64 here.  Parameters
are one flat vector in the order W1 [128x3], b1, W2 [128x128], b2,
W3 [128x128], b3, W4 [3x128], b4 (33,923 values; W is [out, in], row-major).
"""
from __future__ import annotations

import numpy as np

SIZES = (3, 128, 128, 128, 3)


def layout():
    """[(W offset, W shape, b offset, b size)] per layer and the total size."""
    out, off = [], 0
    for i in range(4):
        n_in, n_out = SIZES[i], SIZES[i + 1]
        w_off = off
        off += n_in * n_out
        b_off = off
        off += n_out
        out.append((w_off, (n_out, n_in), b_off, n_out))
    return out, off


LAYOUT, NPARAMS = layout()


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params, round_weights: bool = True):
    """Per-layer (W, b) in FP64; W rounded through bfloat16 when asked."""
    p = np.asarray(params)
    layers = []
    for w_off, shape, b_off, nb in LAYOUT:
        W = p[w_off:w_off + shape[0] * shape[1]].reshape(shape)
        W = bf16_round(W) if round_weights else W.astype(np.float64)
        b = p[b_off:b_off + nb].astype(np.float64)
        layers.append((W, b))
    return layers


def forward(params, x, round_weights: bool = True):
    """Returns the output [B, 3] and the activations (h0 = x, h1, h2, h3)."""
    layers = unpack(params, round_weights)
    h = [np.asarray(x, dtype=np.float64)]
    for i, (W, b) in enumerate(layers):
        z = h[-1] @ W.T + b
        h.append(np.tanh(z) if i < 3 else z)
    return h[-1], h[:-1]


def backward(params, x, dy, round_weights: bool = True):
    """Gradients of sum(dy * y) with respect to the parameters (flat, the weight part
    taken with respect to the rounded weights) and to the input x."""
    layers = unpack(params, round_weights)
    y, hs = forward(params, x, round_weights)
    grad = np.zeros(NPARAMS)
    dz = np.asarray(dy, dtype=np.float64)
    for i in range(3, -1, -1):
        W, _ = layers[i]
        w_off, shape, b_off, nb = LAYOUT[i]
        grad[w_off:w_off + shape[0] * shape[1]] = (dz.T @ hs[i]).ravel()
        grad[b_off:b_off + nb] = dz.sum(axis=0)
        dh = dz @ W
        if i > 0:
            dz = dh * (1.0 - hs[i] ** 2)  # tanh' = 1 - tanh^2
        else:
            dx = dh
    return grad, dx


def mse_loss_grad(y, t):
    """L = mean over batch and outputs of (y - t)^2, and dL/dy."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = y.size
    return float(np.sum((y - t) ** 2) / n), 2.0 * (y - t) / n


def adam_step(params, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of FP32-held parameters, computed in FP64."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases, float32."""
    g = np.random.Generator(np.random.PCG64(seed))
    p = np.empty(NPARAMS, dtype=np.float32)
    for w_off, shape, b_off, nb in LAYOUT:
        s = 1.0 / np.sqrt(shape[1])
        p[w_off:w_off + shape[0] * shape[1]] = g.uniform(-s, s, shape[0] * shape[1])
        p[b_off:b_off + nb] = g.uniform(-s, s, nb)
    return p
