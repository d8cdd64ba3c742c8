"""FP64 oracle of the format selector -- TEST INFRASTRUCTURE ONLY.

The paper's predictor maps static matrix features to the best format label
(Sec. V-A, V-B); features are scaled to [0, 1] with the training set's
per-feature minimum and maximum (Sec. V-B, "Feature Scaling").  Among the
alternative classifiers it evaluates is a multilayer perceptron (Sec. V-D).
The network here is that alternative: 12 -> 64 -> 64 -> 5, ReLU hidden
layers, softmax cross-entropy averaged over the batch, trained with Adam
(Kingma and Ba, 2015).  Shapes: W_l is (fan_in, fan_out), so a layer is
``h @ W + b`` for a row-major batch ``h``.

Written as the plain definitions, one step per line, in float64.
"""
from __future__ import annotations

import numpy as np

LOG_FEATURES = (0, 1, 2, 4, 5, 6, 7, 9, 10)  # size-like: log2(1 + v)
FRAC_FEATURE = 3  # nnz_frac: log2(max(v, 2^-64))


def feature_transform(F):
    """Log step applied before min-max scaling (a documented deviation from
    the paper's plain min-max: sizes span several decades)."""
    F = np.array(F, dtype=np.float64, copy=True)
    F[..., LOG_FEATURES] = np.log2(1.0 + F[..., LOG_FEATURES])
    F[..., FRAC_FEATURE] = np.log2(np.maximum(F[..., FRAC_FEATURE], 2.0 ** -64))
    return F


def minmax_fit(F):
    F = np.asarray(F, dtype=np.float64)
    return F.min(axis=0), F.max(axis=0)


def minmax_apply(F, lo, hi):
    """(v - min) / (max - min) per feature, no clamping; 0 where max == min."""
    F = np.asarray(F, dtype=np.float64)
    span = hi - lo
    out = np.zeros_like(F)
    nz = span > 0
    out[..., nz] = (F[..., nz] - lo[nz]) / span[nz]
    return out


def mlp_forward(params, X):
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3 + b3
    return z, (X, a1, h1, a2, h2)


def softmax(z):
    m = z.max(axis=-1, keepdims=True)
    e = np.exp(z - m)
    return e / e.sum(axis=-1, keepdims=True)


def mlp_loss_and_grads(params, X, labels):
    """Mean softmax cross-entropy over the batch and its gradients
    [dW1, db1, dW2, db2, dW3, db3]."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, dtype=np.float64) for p in params]
    z, (X, a1, h1, a2, h2) = mlp_forward(params, X)
    B = z.shape[0]
    labels = np.asarray(labels, dtype=np.int64)
    m = z.max(axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(z - m).sum(axis=1))
    loss = float(np.mean(lse - z[np.arange(B), labels]))
    dz = softmax(z)
    dz[np.arange(B), labels] -= 1.0
    dz /= B
    dW3 = h2.T @ dz
    db3 = dz.sum(axis=0)
    dh2 = dz @ W3.T
    da2 = dh2 * (a2 > 0.0)
    dW2 = h1.T @ da2
    db2 = da2.sum(axis=0)
    dh1 = da2 @ W2.T
    da1 = dh1 * (a1 > 0.0)
    dW1 = X.T @ da1
    db1 = da1.sum(axis=0)
    return loss, [dW1, db1, dW2, db2, dW3, db3]


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (params, m, v)."""
    newp, newm, newv = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        mi = beta1 * mi + (1.0 - beta1) * g
        vi = beta2 * vi + (1.0 - beta2) * g * g
        mhat = mi / (1.0 - beta1 ** t)
        vhat = vi / (1.0 - beta2 ** t)
        newp.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        newm.append(mi)
        newv.append(vi)
    return newp, newm, newv
