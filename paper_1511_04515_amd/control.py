"""Training data and the training loop of the learned step controller.

Samples come from the solver's own trace records: the features recorded for
accepted step k (computed before its step size was chosen) map to the
targets (m_k, log10 h*_k): the Krylov size the step's first MEVP needed and
the step that its own error estimate says would have met the budget.  Training runs on the GPU through the C ABI
(expri_mlp_*): float32 forward and backward passes and Adam.  This module
only assembles arrays and drives those calls.
"""
from __future__ import annotations

import numpy as np

from .binding import Mlp, MLP_PARAMS

HIDDEN = 64
SIZES = (8, HIDDEN, HIDDEN, 2)


def samples_from_traces(traces, E_rr: float = 1e-6, alpha: float = 0.5, order: float = 3.0):
    """(X, T) float32 arrays from trace dicts (Solver.trace).  X = the eight
    features recorded for step k.  T = (m_k, log10 h*_k): the Krylov size of
    the step's first MEVP and the step that would have met the error budget,
    h*_k = h_k (E_rr / err_k)^(1/order) from the step's own error estimate
    (the estimate scales as h^3), the factor bounded to [1/2, 4] and, after a
    rejection, kept below the rejected trial h_k / alpha.  Steps clipped to
    land on a source corner are left out."""
    X = np.concatenate([tr["feat"] for tr in traces]).astype(np.float64)
    h = np.concatenate([tr["h"] for tr in traces])
    h_try = np.concatenate([tr["h_try"] for tr in traces])
    err = np.concatenate([tr["err"] for tr in traces])
    rej = np.concatenate([tr["rejects"] for tr in traces])
    m = np.concatenate([tr["m"] for tr in traces])
    # steps shortened to land on a source corner say nothing about the step
    # the error budget allows
    landed = (rej == 0) & (h < h_try * (1.0 - 1e-9))
    with np.errstate(divide="ignore"):
        ratio = np.clip((E_rr / np.maximum(err, 1e-300)) ** (1.0 / order), 0.5, 4.0)
    h_star = h * ratio
    h_star = np.where(rej > 0, np.minimum(h_star, 0.9 * h / alpha), h_star)
    T = np.stack([m, np.log10(h_star)], 1)
    keep = np.isfinite(X).all(1) & np.isfinite(T).all(1) & ~landed
    return X[keep].astype(np.float32), T[keep].astype(np.float32)


def initial_params(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, in the flat
    order W1, b1, W2, b2, W3, b3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i in range(len(SIZES) - 1):
        r, c = SIZES[i + 1], SIZES[i]
        parts.append(rng.uniform(-np.sqrt(6.0 / c), np.sqrt(6.0 / c), r * c))
        parts.append(np.zeros(r))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == MLP_PARAMS
    return p


def train(X, T, epochs: int = 20, batch: int = 4096, lr: float = 1e-3, seed: int = 0, log=None):
    """Train on (X, T) with Adam on the GPU; returns (params, norm, losses).
    The samples are shuffled once on the host; minibatches are contiguous
    slices of the shuffled set."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(len(X))
    Xd = torch.from_numpy(np.ascontiguousarray(X[order])).cuda()
    Td = torch.from_numpy(np.ascontiguousarray(T[order])).cuda()
    net = Mlp(initial_params(seed))
    net.fit_norm(Xd, Td)
    losses = []
    n = len(X)
    for ep in range(epochs):
        for lo in range(0, n, batch):
            hi = min(n, lo + batch)
            net.adam_step(Xd[lo:hi], Td[lo:hi], lr=lr)
        loss, _ = net.grad(Xd[:65536], Td[:65536])  # a fixed subset bounds the scratch size
        losses.append(loss)
        if log:
            log(f"epoch {ep}: loss {loss:.4f}")
    params, norm = net.params(), net.norm()
    net.close()
    return params, norm, losses
