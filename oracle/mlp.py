"""Plain numpy oracle of the degree-picker network (TEST INFRASTRUCTURE).

MLP with inputs x (66), three ReLU layers of 128 and 2 linear outputs; one
flat parameter vector, per layer W (out x in, row-major) then b.  Loss
(1/B) sum_i sum_j w_j (out_ij - y_ij)^2.  Forward and the gradient are the
chain rule written out layer by layer, in FP64.
"""
from __future__ import annotations

import numpy as np

DIMS = [66, 128, 128, 128, 2]


def unpack(p: np.ndarray):
    layers, o = [], 0
    for k in range(4):
        n_in, n_out = DIMS[k], DIMS[k + 1]
        W = p[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = p[o:o + n_out]
        o += n_out
        layers.append((W, b))
    assert o == p.size
    return layers


def nparams() -> int:
    return sum(DIMS[k + 1] * DIMS[k] + DIMS[k + 1] for k in range(4))


def init(seed: int = 0, out_scale: float = 0.0) -> np.ndarray:
    """He-normal weights, zero biases; the output layer scaled by out_scale
    (0: the network starts by predicting 0, i.e. the plain rule)."""
    rng = np.random.default_rng(seed)
    parts = []
    for k in range(4):
        n_in, n_out = DIMS[k], DIMS[k + 1]
        W = rng.standard_normal((n_out, n_in)) * np.sqrt(2.0 / n_in)
        if k == 3:
            W *= out_scale
        parts += [W.ravel(), np.zeros(n_out)]
    return np.concatenate(parts)


def forward(p: np.ndarray, X: np.ndarray):
    """Output and the per-layer pre-activations/activations."""
    acts = [np.asarray(X, dtype=np.float64)]
    pre = []
    h = acts[0]
    for k, (W, b) in enumerate(unpack(np.asarray(p, dtype=np.float64))):
        z = h @ W.T + b
        pre.append(z)
        h = np.maximum(z, 0.0) if k < 3 else z
        acts.append(h)
    return h, pre, acts


def loss_and_grad(p: np.ndarray, X: np.ndarray, Y: np.ndarray, w: np.ndarray):
    out, pre, acts = forward(p, X)
    B = X.shape[0]
    d = out - Y
    loss = float(np.sum(w[None, :] * d * d) / B)
    g_out = 2.0 * w[None, :] * d / B
    layers = unpack(np.asarray(p, dtype=np.float64))
    grads = [None] * 4
    delta = g_out
    for k in range(3, -1, -1):
        W, _ = layers[k]
        grads[k] = (delta.T @ acts[k], delta.sum(axis=0))
        if k > 0:
            delta = (delta @ W) * (pre[k - 1] > 0)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat
