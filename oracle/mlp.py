"""The learned step controller's network, written out plainly (test
infrastructure).

A multilayer perceptron 8 -> 64 -> 64 -> 2 with ReLU hidden layers maps the
step features to (m, log10 h) targets; the loss is the mean squared error over
the batch, halved:  L = 1/(2N) sum_n ||y_n - t_n||^2.  Training is Adam
(Kingma & Ba, ICLR 2015) with bias-corrected moments.

Parameters are one flat vector in the order
    W1 (64 x 8, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2)
(4,866 numbers).  Everything here is float64; the GPU trains in float32 and
infers with bfloat16 weights and activations.
"""
from __future__ import annotations

import numpy as np

SIZES = (8, 64, 64, 2)


def n_params(sizes=SIZES) -> int:
    return sum(sizes[i + 1] * sizes[i] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(theta, sizes=SIZES):
    """Views (W1, b1, W2, b2, W3, b3) into the flat parameter vector."""
    out, o = [], 0
    for i in range(len(sizes) - 1):
        r, c = sizes[i + 1], sizes[i]
        out.append(theta[o:o + r * c].reshape(r, c))
        o += r * c
        out.append(theta[o:o + r])
        o += r
    return out


def init(seed: int, sizes=SIZES) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i in range(len(sizes) - 1):
        r, c = sizes[i + 1], sizes[i]
        bound = np.sqrt(6.0 / c)
        parts.append(rng.uniform(-bound, bound, r * c))
        parts.append(np.zeros(r))
    return np.concatenate(parts)


def forward(theta, X, sizes=SIZES):
    """Returns the output and the hidden activations (pre-ReLU kept for the
    backward pass)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, np.float64), sizes)
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    y = a2 @ W3.T + b3
    return y, (X, z1, a1, z2, a2)


def loss(theta, X, T, sizes=SIZES) -> float:
    y, _ = forward(theta, X, sizes)
    return 0.5 * np.sum((y - T) ** 2) / len(X)


def grad(theta, X, T, sizes=SIZES):
    """(loss, dL/dtheta) by the chain rule, layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, np.float64), sizes)
    y, (X, z1, a1, z2, a2) = forward(theta, X, sizes)
    N = len(X)
    dy = (y - T) / N
    gW3 = dy.T @ a2
    gb3 = dy.sum(0)
    dz2 = (dy @ W3) * (z2 > 0)
    gW2 = dz2.T @ a1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    L = 0.5 * np.sum((y - T) ** 2) / N
    return L, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam(theta, g, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def standardize_stats(X, T):
    """Mean and standard deviation (population) of every input feature and
    target over the samples; a constant column gets standard deviation 1.
    The network sees (x - mean) / std and predicts (t - mean) / std."""
    out = []
    for A in (np.asarray(X, np.float64), np.asarray(T, np.float64)):
        mu = A.mean(0)
        sd = np.sqrt(((A - mu) ** 2).mean(0))
        sd[sd == 0.0] = 1.0
        out += [mu, sd]
    return tuple(out)  # (x_mean, x_std, t_mean, t_std)


def to_bf16(a):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as
    float32."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def forward_bf16(theta, X, sizes=SIZES):
    """Inference with bfloat16 weights, inputs and hidden activations and
    float32 sums (products of two bfloat16 values are exact in float32)."""
    W1, b1, W2, b2, W3, b3 = [to_bf16(np.asarray(p, np.float32)) for p in unpack(np.asarray(theta), sizes)]
    h = to_bf16(np.asarray(X, np.float32))
    for W, b, relu in ((W1, b1, True), (W2, b2, True), (W3, b3, False)):
        z = (h.astype(np.float64) @ W.T.astype(np.float64) + b).astype(np.float32)
        h = to_bf16(np.maximum(z, 0.0)) if relu else z
    return h
