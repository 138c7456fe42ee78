"""CPU oracle of the cost-model network -- TEST INFRASTRUCTURE ONLY.

Only tests (and the benchmark's CPU leg) use this module; the GPU library
never imports it.  Plain numpy in fp64:

  forward     a_{l+1} = relu(a_l W_l^T + b_l) for hidden layers, linear last
  loss        L = mean over rows and outputs of (y - t)^2
  backward    dY = 2 (y - t) / (rows * outputs);  dW_l = dY^T a_l;
              db_l = column sums of dY;  dX = (dY W_l) * [a_l > 0]
  adam        m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
              p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

Parameter layout (shared format with the library's flat parameter array):
for each layer l, W_l (out x in, row-major) then b_l (out).
"""
from __future__ import annotations

import numpy as np


def layer_shapes(dims):
    return [(dims[l + 1], dims[l]) for l in range(len(dims) - 1)]


def unpack(params, dims):
    """Split a flat parameter array into [(W_l, b_l)]."""
    p = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    for o, i in layer_shapes(dims):
        W = p[off:off + o * i].reshape(o, i)
        off += o * i
        b = p[off:off + o]
        off += o
        out.append((W, b))
    assert off == p.size, (off, p.size)
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def forward(params, dims, X):
    """All activations [a_0 = X, a_1, ..., a_L] (a_L = network output)."""
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(params, dims)
    for l, (W, b) in enumerate(layers):
        z = acts[-1] @ W.T + b
        acts.append(np.maximum(z, 0.0) if l < len(layers) - 1 else z)
    return acts


def mse(Y, T):
    Y = np.asarray(Y, np.float64)
    T = np.asarray(T, np.float64)
    return float(np.mean((Y - T) ** 2))


def loss_grad(params, dims, X, T):
    """(loss, flat gradient) of the mean squared error."""
    layers = unpack(params, dims)
    acts = forward(params, dims, X)
    T = np.asarray(T, np.float64)
    Y = acts[-1]
    loss = float(np.mean((Y - T) ** 2))
    d = 2.0 * (Y - T) / Y.size
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (d.T @ acts[l], d.sum(axis=0))
        if l > 0:
            d = (d @ W) * (acts[l] > 0)
    return loss, pack(grads)


def adam_step(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step count t starts at 1); returns (params, m, v)."""
    p = np.asarray(params, np.float64)
    g = np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def n_params(dims):
    return sum(o * i + o for o, i in layer_shapes(dims))
