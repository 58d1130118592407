"""FP64 reference of the planner's cost-model network (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by tests to check the library's HIP training
kernels; it shares no code with them.  The network is the one the library
documents: inputs normalised as (x - xmean) / xstd, three hidden layers of H
SiLU units (silu(z) = z sigmoid(z)), one linear output; the loss is the mean
squared error between the output and the normalised target
(y - ymean) / ystd.  The parameter vector is W1[NF][H], b1[H], W2[H][H],
b2[H], W3[H][H], b3[H], W4[H], b4, then xmean[NF], xstd[NF], ymean, ystd.

The gradient is the textbook chain rule written out layer by layer; its pin
is a central finite difference of ``loss`` (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np


def unpack(params, nf: int, h: int):
    p = np.asarray(params, dtype=np.float64)
    shapes = [(nf, h), (h,), (h, h), (h,), (h, h), (h,), (h, 1), (1,)]
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    xmean = p[o:o + nf]
    xstd = p[o + nf:o + 2 * nf]
    ymean, ystd = p[o + 2 * nf], p[o + 2 * nf + 1]
    return out, (xmean, xstd, ymean, ystd), o


def _silu(z):
    return z / (1.0 + np.exp(-z))


def _dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, nf: int, h: int):
    """Normalised prediction and the per-layer (input, pre-activation) pairs."""
    W, (xm, xs, _, _), _ = unpack(params, nf, h)
    a = (np.asarray(X, dtype=np.float64) - xm) / xs
    cache = []
    for l in range(4):
        z = a @ W[2 * l] + W[2 * l + 1]
        cache.append((a, z))
        a = _silu(z) if l < 3 else z
    return a[:, 0], cache


def loss(params, X, y, nf: int, h: int) -> float:
    _, (_, _, ym, ys), _ = unpack(params, nf, h)
    yhat, _ = forward(params, X, nf, h)
    t = (np.asarray(y, dtype=np.float64) - ym) / ys
    return float(np.mean((yhat - t) ** 2))


def grad(params, X, y, nf: int, h: int):
    """Gradient of ``loss`` with respect to the network parameters (not the normalisation)."""
    W, (_, _, ym, ys), nnet = unpack(params, nf, h)
    yhat, cache = forward(params, X, nf, h)
    n = yhat.shape[0]
    t = (np.asarray(y, dtype=np.float64) - ym) / ys
    d = (2.0 / n) * (yhat - t)[:, None]      # d loss / d output
    grads = [None] * 8
    for l in range(3, -1, -1):
        a_in, z = cache[l]
        dz = d if l == 3 else d * _dsilu(z)
        grads[2 * l] = a_in.T @ dz
        grads[2 * l + 1] = dz.sum(axis=0)
        d = dz @ W[2 * l].T
    return np.concatenate([g.ravel() for g in grads]), nnet


def predict_log_ms(params, X, nf: int, h: int):
    """De-normalised prediction (log ms)."""
    _, (_, _, ym, ys), _ = unpack(params, nf, h)
    yhat, _ = forward(params, X, nf, h)
    return yhat * ys + ym
