"""FP64 reference of the screener network (TEST INFRASTRUCTURE ONLY).

Three dense layers 32 -> 128 -> 128 -> 4 with ReLU after the first two and a sigmoid
output, binary cross-entropy averaged over the batch and the 4 outputs, and Adam.
The flat parameter layout is, per layer, W (in x out, row-major) then b (out).
"""
from __future__ import annotations

import numpy as np

LAYERS = [(32, 128), (128, 128), (128, 4)]


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for i, o in LAYERS:
        W = theta[k:k + i * o].reshape(i, o)
        k += i * o
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    assert k == theta.size
    return out


def forward(theta, X):
    """Returns (pre-activations per layer, activations per layer, probabilities)."""
    layers = unpack(theta)
    a = np.asarray(X, dtype=np.float64)
    acts, pres = [a], []
    for li, (W, b) in enumerate(layers):
        z = a @ W + b
        pres.append(z)
        a = np.maximum(z, 0.0) if li < len(layers) - 1 else z
        acts.append(a)
    logits = pres[-1]
    return pres, acts, 1.0 / (1.0 + np.exp(-logits))


def loss(theta, X, Y) -> float:
    pres, _, _ = forward(theta, X)
    z = pres[-1]
    Y = np.asarray(Y, dtype=np.float64)
    # -[y log s(z) + (1-y) log(1-s(z))] = max(z,0) - z y + log(1 + e^{-|z|})
    return float(np.mean(np.maximum(z, 0) - z * Y + np.log1p(np.exp(-np.abs(z)))))


def loss_and_grad(theta, X, Y):
    """Backpropagation: dL/dz_out = (sigmoid(z) - y) / (B * 4), then through the layers."""
    pres, acts, p = forward(theta, X)
    Y = np.asarray(Y, dtype=np.float64)
    B = Y.shape[0]
    layers = unpack(theta)
    dz = (p - Y) / (B * Y.shape[1])
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads[li] = (acts[li].T @ dz, dz.sum(axis=0))
        if li > 0:
            da = dz @ W.T
            dz = da * (pres[li - 1] > 0)
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1]]) for g in grads])
    return loss(theta, X, Y), flat


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; t counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
