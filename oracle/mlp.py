"""ACA-rank predictor network (oracle, float64).

Not a method of the paper: a small learned model that predicts the ACA rank of
a (far block, frequency) pair so that work tiles can be sized before the
adaptive ACA runs (the ACA still decides the rank).

  features  x = [diam |s| / c, dist Re(s) / c, dist |Im(s)| / c,
                 log2 |I|, log2 |J|], standardised with the training-set mean
                 and standard deviation
  network   5 -> 64 -> 64 -> 1, tanh hidden layers, linear output
  target    log(1 + rank); loss = mean squared error (1/2 mean (y - t)^2)
  optimiser Adam(lr, beta1, beta2, eps = 1e-8) with bias correction
  init      Glorot-uniform weights, zero biases

Parameter vector layout (shared by the library's get/set calls):
  W1 (64, 5), b1 (64), W2 (64, 64), b2 (64), W3 (1, 64), b3 (1), row-major.
"""
from __future__ import annotations

import numpy as np

SIZES = [(64, 5), (64,), (64, 64), (64,), (1, 64), (1,)]
N_PARAMS = sum(int(np.prod(s)) for s in SIZES)


def unpack(theta):
    out, o = [], 0
    for s in SIZES:
        k = int(np.prod(s))
        out.append(np.asarray(theta[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def glorot_init(seed: int = 0):
    rng = np.random.default_rng(seed)
    parts = []
    for s in SIZES:
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, size=s))
        else:
            parts.append(np.zeros(s))
    return pack(parts)


def forward(theta, X):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    a1 = X @ W1.T + b1
    h1 = np.tanh(a1)
    a2 = h1 @ W2.T + b2
    h2 = np.tanh(a2)
    y = (h2 @ W3.T + b3)[:, 0]
    return y, (X, h1, h2)


def loss_and_grad(theta, X, t):
    """Loss 1/2 mean (y - t)^2 and its gradient by back-propagation."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (X, h1, h2) = forward(theta, X)
    B = len(t)
    e = (y - t) / B                                  # dL/dy
    loss = 0.5 * np.sum((y - t) ** 2) / B
    gW3 = e[None, :] @ h2                            # (1, 64)
    gb3 = np.array([e.sum()])
    d2 = (e[:, None] @ W3) * (1.0 - h2 ** 2)         # (B, 64)
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    d1 = (d2 @ W2) * (1.0 - h1 ** 2)
    gW1 = d1.T @ X
    gb1 = d1.sum(0)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, grad, m, v, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(diam, dist, s, c, nI, nJ):
    """Raw (unstandardised) features of (block, frequency) pairs; all inputs broadcast."""
    s = np.asarray(s, dtype=np.complex128)
    return np.stack([np.asarray(diam) * np.abs(s) / c,
                     np.asarray(dist) * s.real / c,
                     np.asarray(dist) * np.abs(s.imag) / c,
                     np.log2(np.asarray(nI, dtype=np.float64)),
                     np.log2(np.asarray(nJ, dtype=np.float64))], axis=-1)


def capacity(pred_log1p_rank, floor: int = 4, multiple: int = 4):
    """Tile capacity from a predicted log(1 + r): ceil(1.25 r) + 2, rounded up
    to a multiple of ``multiple``, at least ``floor``."""
    r = np.maximum(np.expm1(np.asarray(pred_log1p_rank, dtype=np.float64)), 0.0)
    cap = np.ceil(1.25 * r) + 2
    cap = np.ceil(cap / multiple) * multiple
    return np.maximum(cap, floor).astype(np.int64)
