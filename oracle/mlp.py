"""FP64 NumPy oracle of the prefill MLP (test infrastructure only).

The network: x (8 features) -> tanh(x W1 + b1) -> tanh(h1 W2 + b2) -> h2 W3 + b3
= (u, v), with 64 hidden units.  Parameters are held as one flat vector in the
layout W1[8][64] b1[64] W2[64][64] b2[64] W3[64][2] b3[2] (row-major "in x out").
Every routine here is the textbook definition, in float64, evaluated on the
bfloat16-rounded weights the device uses.  The backward pass is pinned against
central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

IN, H, OUT = 8, 64, 2
SIZES = [("W1", (IN, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, OUT)), ("b3", (OUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, at = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = flat[at:at + n].reshape(shape)
        at += n
    return out


def bf16_round(x32: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round to nearest, ties to even."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint16)
    nan = (u & np.uint64(0x7F800000)) == np.uint64(0x7F800000)
    nan &= (u & np.uint64(0x007FFFFF)) != 0
    r[nan] = ((u[nan] >> np.uint64(16)) | np.uint64(0x40)).astype(np.uint16)
    return r


def bf16_to_f64(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def forward(params, x):
    """Returns y (B, 2) and the cache (h1, h2)."""
    p = unpack(params)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(x @ p["W1"] + p["b1"])
    h2 = np.tanh(h1 @ p["W2"] + p["b2"])
    y = h2 @ p["W3"] + p["b3"]
    return y, (h1, h2)


def backward(params, x, cache, dy):
    """Gradient of sum(dy * y) with respect to the flat parameter vector."""
    p = unpack(params)
    x = np.asarray(x, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    h1, h2 = cache
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dz2 = (dy @ p["W3"].T) * (1.0 - h2 * h2)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * (1.0 - h1 * h1)
    dW1 = x.T @ dz1
    db1 = dz1.sum(axis=0)
    return np.concatenate([g.ravel() for g in (dW1, db1, dW2, db2, dW3, db3)])


def loss_and_dy(y, target, weight):
    """Weighted mean squared error over rows and both outputs, and dL/dy."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    w = np.asarray(weight, dtype=np.float64)
    wn = w / w.sum()
    r = y - t
    loss = float((wn[:, None] * r * r).sum())
    return loss, 2.0 * wn[:, None] * r


def adam_step(w, m, v, g, lr, b1, b2, eps, wd, step):
    """One Adam step with decoupled weight decay (float64)."""
    w = np.asarray(w, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1**step)
    vh = v / (1.0 - b2**step)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v
