"""FP64 NumPy oracle of the smoothing-length network (test infrastructure).

The network is not part of the paper; it proposes a starting support radius
for the smoothing-length iteration of eqs. (hi) and (thacker). Its shape is
8 -> 64 -> 64 -> 1 with exact-erf GELU activations:

    z1 = W1 f + b1,  a1 = gelu(z1),  z2 = W2 a1 + b2,  a2 = gelu(z2),
    y  = w3 . a2 + b3,   gelu(x) = x/2 (1 + erf(x / sqrt 2)).

Training minimises the mean squared error mean_b (y_b - t_b)^2 with Adam
(beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected). Parameters are kept in
one flat vector in the order W1 (64x8, row-major), b1, W2 (64x64), b2, w3,
b3 — 4801 values. Everything here is plain FP64 loops over layers with a
hand-written backward pass, so it can be checked by finite differences.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

D_IN, D_H = 8, 64
SHAPES = (("W1", (D_H, D_IN)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
          ("w3", (D_H,)), ("b3", (1,)))
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray) -> dict:
    out, k = {}, 0
    for name, shp in SHAPES:
        sz = int(np.prod(shp))
        out[name] = theta[k:k + sz].reshape(shp)
        k += sz
    return out


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta: np.ndarray, f: np.ndarray, keep: bool = False):
    """f: (B, 8) -> y: (B,). With keep=True also returns the activations."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    f = np.asarray(f, dtype=np.float64)
    z1 = f @ p["W1"].T + p["b1"]
    a1 = gelu(z1)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = gelu(z2)
    y = a2 @ p["w3"] + p["b3"][0]
    if keep:
        return y, (f, z1, a1, z2, a2)
    return y


def loss(theta, f, t):
    y = forward(theta, f)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def backward(theta: np.ndarray, f: np.ndarray, t: np.ndarray):
    """(loss, gradient of the loss w.r.t. the flat parameter vector)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    y, (f, z1, a1, z2, a2) = forward(theta, f, keep=True)
    B = f.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    dy = 2.0 * r / B
    g = {}
    g["w3"] = a2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, p["w3"]) * gelu_grad(z2)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(0)
    da1 = dz2 @ p["W2"]
    dz1 = da1 * gelu_grad(z1)
    g["W1"] = dz1.T @ f
    g["b1"] = dz1.sum(0)
    flat = np.concatenate([g[name].ravel() for name, _ in SHAPES])
    return float(np.mean(r * r)), flat


class Adam:
    """Bias-corrected Adam on the flat parameter vector."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * grad
        self.v = self.b2 * self.v + (1.0 - self.b2) * grad * grad
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)
