"""Cost-model network in float64 -- TEST INFRASTRUCTURE ONLY.

The learned cost model is not in the paper: it stands in for the auto-tuning
step the paper leaves open (program parameters "can be deduced, for instance,
by auto-tuning", Section 1).  This module is the plain definition of what the
HIP kernels compute, in float64 and numpy:

* network: x (IN = 13 features) -> h1 = relu(W1 x + b1) (64) -> h2 =
  relu(W2 h1 + b2) (64) -> y = W3 h2 + b3 (1); 5121 parameters;
* loss: mean squared error L = (1/n) sum_r (y_r - t_r)^2;
* gradients: the chain rule written out layer by layer (relu'(z) = [z > 0]);
* Adam (Kingma and Ba, 2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
  mhat = m / (1-b1^t), vhat = v / (1-b2^t), p <- p - lr mhat / (sqrt(vhat) + eps).

Parameter order (also the flat layout): W1 (64x13, row-major), b1 (64),
W2 (64x64), b2 (64), W3 (1x64), b3 (1).
"""
from __future__ import annotations

import numpy as np

IN, H1, H2, OUT = 13, 64, 64, 1
SHAPES = (("W1", (H1, IN)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)),
          ("W3", (OUT, H2)), ("b3", (OUT,)))
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(flat: np.ndarray) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp)
        o += n
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def forward(p: dict, X: np.ndarray):
    """Returns (y, cache) for a batch X of shape (n, IN); y has shape (n,)."""
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ p["W3"].T + p["b3"])[:, 0]
    return y, (X, z1, h1, z2, h2)


def mse(y: np.ndarray, t: np.ndarray) -> float:
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d))


def backward(p: dict, cache, y: np.ndarray, t: np.ndarray) -> dict:
    """Gradients of the mean squared error with respect to every parameter."""
    X, z1, h1, z2, h2 = cache
    n = X.shape[0]
    dy = (2.0 / n) * (np.asarray(y, np.float64) - np.asarray(t, np.float64))   # dL/dy, (n,)
    dy = dy[:, None]
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return g


def loss_and_grad(flat: np.ndarray, X, t):
    p = unflatten(flat)
    y, cache = forward(p, X)
    return mse(y, t), flatten(backward(p, cache, y, t))


class Adam:
    def __init__(self, n: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, params: np.ndarray, grad: np.ndarray) -> np.ndarray:
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * grad
        self.v = self.b2 * self.v + (1.0 - self.b2) * grad * grad
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        return params - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def init_params(seed: int) -> np.ndarray:
    """He-uniform initialisation (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-bound, bound, size=shp)
        else:
            p[name] = np.zeros(shp)
    return flatten(p)
