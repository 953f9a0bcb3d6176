"""FP64 CPU oracle of the learned surrogate (the MLP of the batched sweep).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP training and
inference kernels; shares no code with them.

The network is the one the surrogate layer specifies (not a part of the
paper's method): 5 inputs -> 256 -> 256 -> 256 -> 2 outputs, fully connected,
GELU after each hidden layer in its exact form
GELU(x) = x Phi(x) = x (1 + erf(x / sqrt 2)) / 2 (Hendrycks and Gimpel, 2016),
trained on a masked mean squared error with Adam (Kingma and Ba, 2015;
bias-corrected moment estimates).  Parameters are laid out per layer as the
weight matrix W[in][out] (row-major) followed by the bias b[out].

`bf16=True` evaluates the method as the GPU path defines it: the weights and
each layer's input rounded to bfloat16 (round to nearest even), products
accumulated exactly (here in FP64), biases, activations and the loss in full
precision.  With `bf16=False` everything is FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

LAYERS = [5, 256, 256, 256, 2]


def n_params(layers=LAYERS) -> int:
    return sum(a * b + b for a, b in zip(layers[:-1], layers[1:]))


def unpack(theta: np.ndarray, layers=LAYERS):
    """Views (W, b) per layer of a flat parameter vector."""
    out, o = [], 0
    for a, b in zip(layers[:-1], layers[1:]):
        W = theta[o:o + a * b].reshape(a, b)
        o += a * b
        bias = theta[o:o + b]
        o += b
        out.append((W, bias))
    return out


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta: np.ndarray, X: np.ndarray, bf16: bool = False, layers=LAYERS):
    """Outputs [B][2] and the per-layer caches (input a, pre-activation z)."""
    a = np.asarray(X, dtype=np.float64)
    cache = []
    params = unpack(np.asarray(theta, dtype=np.float64), layers)
    for k, (W, b) in enumerate(params):
        ain = round_bf16(a) if bf16 else a
        Wq = round_bf16(W) if bf16 else W
        z = ain @ Wq + b
        cache.append((ain, Wq, z))
        a = gelu(z) if k < len(params) - 1 else z
    return a, cache


def loss(theta, X, T, M, bf16: bool = False, layers=LAYERS) -> float:
    """Masked MSE: sum over samples and outputs of M (Y - T)^2, divided by the
    number of unmasked entries."""
    Y, _ = forward(theta, X, bf16, layers)
    return float(np.sum(M * (Y - T) ** 2) / max(np.sum(M), 1.0))


def gradient(theta, X, T, M, bf16: bool = False, layers=LAYERS) -> np.ndarray:
    """d loss / d theta by the chain rule through the layers (backpropagation).
    In bf16 mode the weight gradient is taken with respect to the master
    (unrounded) weights through the rounding (straight-through), i.e. using
    the rounded operands of the forward pass, and the back-propagated signal
    dz enters both of its products (dz W^T and a^T dz) rounded to bfloat16 as
    well, as the GPU path's matrix-core operands are; the bias gradient sums
    the unrounded dz."""
    Y, cache = forward(theta, X, bf16, layers)
    denom = max(float(np.sum(M)), 1.0)
    dz = 2.0 * M * (Y - T) / denom
    grads = []
    for k in range(len(cache) - 1, -1, -1):
        ain, Wq, z = cache[k]
        if k < len(cache) - 1:
            dz = dz * gelu_grad(z)
        dzq = round_bf16(dz) if bf16 else dz
        dW = ain.T @ dzq
        db = dz.sum(axis=0)
        grads.append((dW, db))
        if k > 0:
            dz = dzq @ Wq.T     # gradient w.r.t. the previous layer's output
    g = []
    for dW, db in reversed(grads):
        g.append(dW.ravel())
        g.append(db)
    return np.concatenate(g)


def adam_step(theta, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step count t >= 1), returning new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int, layers=LAYERS) -> np.ndarray:
    """Deterministic initial parameters: W ~ U(-1, 1) sqrt(6 / (in + out)) (Glorot
    uniform), b = 0, from numpy's seeded generator (tests pass the same vector to
    the GPU path)."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(layers[:-1], layers[1:]):
        lim = math.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(np.zeros(b))
    return np.concatenate(parts)
