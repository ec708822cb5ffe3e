"""Oracle of the learned nudging warm start: a 3-layer perceptron
n_in -> n_hidden -> n_hidden -> n_out with ReLU, its mean-squared-error
gradient and Adam.  TEST INFRASTRUCTURE ONLY (same rules as the rest of
``oracle/``): plain numpy, shares nothing with the GPU library.

Two paths:
* ``*_f64``: exact arithmetic in float64 (the definition of the network);
* ``*_bf16``: the mixed-precision definition the GPU implements -- the
  quantities listed below are rounded to bfloat16 (round to nearest, ties to
  even, from float32), every product sum is accumulated exactly (float64
  here; float32 on the GPU, within the tolerance the tests state).

Rounding points of the mixed-precision path: the features X, the weight
matrices W1, W2, W3 (from the float32 master copy), the activations H1, H2 and
the back-propagated errors dY, dZ2, dZ1.  Biases, pre-activations Z, outputs
Y, gradients and Adam state are float32 on the GPU.

Parameter vector layout (float32 master copy, also used for the gradient and
the Adam moments): W1 [H][F], b1 [H], W2 [H][H], b2 [H], W3 [O][H], b3 [O]
(row-major, out x in).
"""
from __future__ import annotations

import numpy as np


def layout(n_in: int, n_hidden: int, n_out: int):
    """Offsets and shapes of the parameter vector."""
    F, H, O = n_in, n_hidden, n_out
    parts = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (O, H)),
             ("b3", (O,))]
    out, off = {}, 0
    for name, shape in parts:
        size = int(np.prod(shape))
        out[name] = (off, shape)
        off += size
    return out, off


def unpack(theta, n_in, n_hidden, n_out):
    lay, _ = layout(n_in, n_hidden, n_out)
    return {k: np.asarray(theta[o:o + int(np.prod(s))]).reshape(s) for k, (o, s) in lay.items()}


def pack(parts, n_in, n_hidden, n_out):
    lay, total = layout(n_in, n_hidden, n_out)
    theta = np.zeros(total)
    for k, (o, s) in lay.items():
        theta[o:o + int(np.prod(s))] = np.asarray(parts[k], dtype=np.float64).ravel()
    return theta


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) from float32; returned as
    float64 values.  NaN stays NaN."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), u | 0x00400000, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of bf16(x)."""
    return (np.asarray(bf16(x), dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).astype(np.uint32).view(np.float32).astype(
        np.float64)


def f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float64)


# --------------------------------------------------------------------------- float64 path
def forward_f64(theta, X, dims):
    p = unpack(theta, *dims)
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ p["W3"].T + p["b3"]
    return Y, (Z1, H1, Z2, H2)


def loss_grad_f64(theta, X, T, dims):
    """Mean squared error over all B x O outputs and its gradient."""
    p = unpack(theta, *dims)
    Y, (Z1, H1, Z2, H2) = forward_f64(theta, X, dims)
    B, O = Y.shape
    R = Y - T
    loss = float(np.sum(R * R) / (B * O))
    dY = 2.0 * R / (B * O)
    g = {"W3": dY.T @ H2, "b3": dY.sum(axis=0)}
    dZ2 = (dY @ p["W3"]) * (Z2 > 0)
    g["W2"], g["b2"] = dZ2.T @ H1, dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * (Z1 > 0)
    g["W1"], g["b1"] = dZ1.T @ X, dZ1.sum(axis=0)
    return loss, pack(g, *dims)


# --------------------------------------------------------------------------- mixed precision
def forward_bf16(theta, X, dims):
    """X: feature values (rounded to bf16 here).  Returns Y (float32 values)
    and the saved activations."""
    p = unpack(f32(theta), *dims)
    Xb = bf16(X)
    W1, W2, W3 = bf16(p["W1"]), bf16(p["W2"]), bf16(p["W3"])
    Z1 = f32(Xb @ W1.T + p["b1"])
    H1 = bf16(np.maximum(Z1, 0.0))
    Z2 = f32(H1 @ W2.T + p["b2"])
    H2 = bf16(np.maximum(Z2, 0.0))
    Y = f32(H2 @ W3.T + p["b3"])
    return Y, (Xb, Z1, H1, Z2, H2)


def loss_grad_bf16(theta, X, T, dims):
    p = unpack(f32(theta), *dims)
    W2, W3 = bf16(p["W2"]), bf16(p["W3"])
    Y, (Xb, Z1, H1, Z2, H2) = forward_bf16(theta, X, dims)
    B, O = Y.shape
    R = Y - f32(T)
    loss = float(np.sum(R * R) / (B * O))
    dYf = f32(2.0 * R / (B * O))
    dY = bf16(dYf)
    g = {"W3": f32(dY.T @ H2), "b3": f32(dYf.sum(axis=0))}
    dZ2f = f32((dY @ W3) * (Z2 > 0))
    dZ2 = bf16(dZ2f)
    g["W2"], g["b2"] = f32(dZ2.T @ H1), f32(dZ2f.sum(axis=0))
    dZ1f = f32((dZ2 @ W2) * (Z1 > 0))
    dZ1 = bf16(dZ1f)
    g["W1"], g["b1"] = f32(dZ1.T @ Xb), f32(dZ1f.sum(axis=0))
    return loss, pack(g, *dims)


# --------------------------------------------------------------------------- Adam
def adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, Algorithm 1) at step t >= 1; returns new
    (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
