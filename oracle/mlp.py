"""FP64 reference of the learned cost model (test infrastructure only).

A multilayer perceptron d -> h (L hidden layers, ReLU) -> 1, mean-squared
error, and Adam (Kingma and Ba, 2015), written with plain numpy float64
matrix products. The flat parameter layout matches the GPU library: for each
layer, the row-major (in x out) weight matrix followed by its out biases.
"""
from __future__ import annotations

import numpy as np


def layout(d: int, h: int, L: int):
    """[(w_off, b_off, in, out)] per layer (L hidden layers + the output layer)."""
    out, off = [], 0
    for l in range(L + 1):
        i = d if l == 0 else h
        o = 1 if l == L else h
        out.append((off, off + i * o, i, o))
        off += i * o + o
    return out, off


def unpack(params, d, h, L):
    lay, _ = layout(d, h, L)
    p = np.asarray(params, dtype=np.float64)
    return [(p[w:w + i * o].reshape(i, o), p[b:b + o]) for (w, b, i, o) in lay]


def forward(params, X, d, h, L):
    """Prediction and the activations of every layer (input first)."""
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(params, d, h, L)
    for l, (W, b) in enumerate(layers):
        z = acts[-1] @ W + b
        acts.append(np.maximum(z, 0.0) if l < L else z)
    return acts[-1][:, 0], acts


def loss_grad(params, X, y, d, h, L):
    """MSE loss and its gradient with respect to the flat parameter vector.
    The ReLU derivative is taken as 1 where the output is > 0, else 0."""
    pred, acts = forward(params, X, d, h, L)
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    loss = float(np.mean((pred - y) ** 2))
    lay, total = layout(d, h, L)
    layers = unpack(params, d, h, L)
    g = np.zeros(total, dtype=np.float64)
    delta = (2.0 * (pred - y) / n)[:, None]            # dLoss / d output (n x 1)
    for l in range(L, -1, -1):
        w_off, b_off, i, o = lay[l]
        g[w_off:w_off + i * o] = (acts[l].T @ delta).ravel()
        g[b_off:b_off + o] = delta.sum(axis=0)
        if l > 0:
            delta = (delta @ layers[l][0].T) * (acts[l] > 0)
    return loss, g


def adam(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with bias correction; returns new (params, m, v)."""
    p = np.asarray(params, dtype=np.float64)
    g = np.asarray(grads, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
