"""ORACLE -- test infrastructure only.

Plain FP64 numpy reference of the parameter predictor: a multilayer perceptron
that maps Chebyshev (KPM) moments of the matrix plus the scaled search interval
to the filter degree and subspace size.  The paper motivates the moments as a
cheap description of the spectrum (Sect. 2: the filter's dot products give the
KPM moments, the density of states and the eigenvalue count) and leaves the
choice of n_p and n_s to heuristics (Sect. 2, Sect. 2.1); the predictor and its
training are a reading added on top, stated here:

  features x (258) = 256 normalised moments mu~_0..mu~_255 and [a~, b~]
  h1 = relu(W1 x + b1)          W1: 128 x 258
  h2 = relu(W2 h1 + b2)         W2: 128 x 128
  y  = W3 h2 + b3               W3:   2 x 128
  loss = (1 / (2 B)) sum_batch ||y - t||^2   (t: standardised log n_p, log n_s)
  Adam (Kingma and Ba) with bias correction.

Parameters are one flat vector in the order W1, b1, W2, b2, W3, b3, each weight
matrix row-major (output index slowest).
"""
from __future__ import annotations

import numpy as np

D_IN, D_H, D_OUT = 258, 128, 2
SHAPES = [(D_H, D_IN), (D_H,), (D_H, D_H), (D_H,), (D_OUT, D_H), (D_OUT,)]


def param_count(shapes=SHAPES) -> int:
    return int(sum(np.prod(s) for s in shapes))


def unflatten(theta: np.ndarray, shapes=SHAPES):
    out, at = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(theta[at:at + k].reshape(s))
        at += k
    return out


def init_params(seed: int, shapes=SHAPES) -> np.ndarray:
    """He-normal weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in shapes:
        if len(s) == 2:
            parts.append(rng.standard_normal(s).ravel() * np.sqrt(2.0 / s[1]))
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def forward(theta: np.ndarray, X: np.ndarray, shapes=SHAPES):
    """X: (B, D_IN) -> y: (B, D_OUT); also returns the pre-activations."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, shapes)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    return y, (z1, h1, z2, h2)


def loss(theta: np.ndarray, X: np.ndarray, T: np.ndarray, shapes=SHAPES) -> float:
    y, _ = forward(theta, X, shapes)
    return float(0.5 * np.sum((y - T) ** 2) / X.shape[0])


def gradient(theta: np.ndarray, X: np.ndarray, T: np.ndarray, shapes=SHAPES):
    """(loss, d loss / d theta) by the chain rule, layer by layer."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, shapes)
    B = X.shape[0]
    y, (z1, h1, z2, h2) = forward(theta, X, shapes)
    dy = (y - T) / B
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return float(0.5 * np.sum((y - T) ** 2) / B), g


def adam(theta, g, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
