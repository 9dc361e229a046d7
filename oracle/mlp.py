"""MLP codec-selector oracle in fp64 numpy -- TEST INFRASTRUCTURE ONLY.

Network 8 -> 64 (ReLU) -> 64 (ReLU) -> 35 that maps the eight fp16 block
features to a score per codec class (0 = bitmap, 1..33 = bit-pack width 0..32,
34 = PFOR).  The paper picks one codec offline from its comparison tables
(the experimental-performance section); a per-block learned choice is this
project's addition, so every rounding point below is this project's reading:

inference / forward
    weights rounded to fp16 (round to nearest even) from the fp32 master copy;
    inputs are fp16; each hidden layer is  h = fp16(relu(W_h x + b)),  with the
    bias kept in fp32; logits  z = W3_h h2 + b3  stay unrounded.
training
    mean softmax cross-entropy against the exhaustive class; the backward pass
    treats each fp16 rounding as the identity (straight-through) and uses the
    rounded values wherever the forward pass used them; Adam (Kingma & Ba):
    beta1 0.9, beta2 0.999, eps 1e-8 with bias correction.

``rounding=False`` drops every fp16 rounding; that exact-arithmetic network is
the one the finite-difference test pins.
Flat parameter order: W1[64][8] b1[64] W2[64][64] b2[64] W3[35][64] b3[35].
"""
from __future__ import annotations

import numpy as np

DIMS = (8, 64, 64, 35)


def n_params() -> int:
    return sum(DIMS[i] * DIMS[i + 1] + DIMS[i + 1] for i in range(3))


def unpack(theta: np.ndarray):
    theta = np.asarray(theta, np.float64)
    out, k = [], 0
    for i in range(3):
        fi, fo = DIMS[i], DIMS[i + 1]
        W = theta[k:k + fo * fi].reshape(fo, fi)
        k += fo * fi
        b = theta[k:k + fo]
        k += fo
        out.append((W, b))
    assert k == theta.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def f16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest fp16 value (ties to even), returned as fp64."""
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def features_to_f64(feat_bits: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(feat_bits, np.uint16).view(np.float16).astype(np.float64)


def forward(theta, X, rounding: bool = True):
    """X: fp64 [N, 8] (values of fp16 features).  Returns logits and a cache."""
    (W1, b1), (W2, b2), (W3, b3) = unpack(theta)
    r = f16 if rounding else (lambda a: np.asarray(a, np.float64))
    W1h, W2h, W3h = r(W1), r(W2), r(W3)
    z1 = X @ W1h.T + b1
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ W2h.T + b2
    h2 = r(np.maximum(z2, 0.0))
    z3 = h2 @ W3h.T + b3
    cache = (X, W1h, W2h, W3h, z1, h1, z2, h2)
    return z3, cache


def loss_and_grad(theta, X, y, rounding: bool = True):
    """Mean softmax cross-entropy and its gradient (straight-through at the
    fp16 rounding points)."""
    z3, (X, W1h, W2h, W3h, z1, h1, z2, h2) = forward(theta, X, rounding)
    N = X.shape[0]
    y = np.asarray(y, np.int64)
    zmax = z3.max(axis=1, keepdims=True)
    ez = np.exp(z3 - zmax)
    ssum = ez.sum(axis=1, keepdims=True)
    logp = z3 - zmax - np.log(ssum)
    loss = -logp[np.arange(N), y].mean()
    g3 = ez / ssum
    g3[np.arange(N), y] -= 1.0
    g3 /= N
    dW3 = g3.T @ h2
    db3 = g3.sum(axis=0)
    d2 = (g3 @ W3h) * (z2 > 0)
    dW2 = d2.T @ h1
    db2 = d2.sum(axis=0)
    d1 = (d2 @ W2h) * (z1 > 0)
    dW1 = d1.T @ X
    db1 = d1.sum(axis=0)
    return float(loss), pack([(dW1, db1), (dW2, db2), (dW3, db3)])


def loss_only(theta, X, y, rounding: bool = True) -> float:
    return loss_and_grad(theta, X, y, rounding)[0]


def predict(theta, X) -> np.ndarray:
    """Argmax class per row; ties go to the lowest index; rows with a NaN
    logit give 255 (caller falls back to the exhaustive class)."""
    z3, _ = forward(theta, X, True)
    cls = np.argmax(z3, axis=1).astype(np.int64)  # first maximum on ties
    cls[np.isnan(z3).any(axis=1)] = 255
    return cls.astype(np.uint8)


class Adam:
    def __init__(self, n: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.beta1 * self.m + (1 - self.beta1) * g
        self.v = self.beta2 * self.v + (1 - self.beta2) * g * g
        mhat = self.m / (1 - self.beta1 ** self.t)
        vhat = self.v / (1 - self.beta2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def finite_difference(theta, X, y, idx, h=1e-6):
    """Central differences of the exact-arithmetic loss at parameters idx."""
    out = np.empty(len(idx))
    for t, i in enumerate(idx):
        tp = np.array(theta, np.float64)
        tm = np.array(theta, np.float64)
        tp[i] += h
        tm[i] -= h
        out[t] = (loss_only(tp, X, y, False) - loss_only(tm, X, y, False)) / (2 * h)
    return out
