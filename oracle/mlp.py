"""FP64 reference for the learned rank estimator (forward, backward, Adam).

TEST INFRASTRUCTURE ONLY (see oracle.py).

The estimator maps a per-(user, query) feature vector x (18 values: the
query score over the user norm, the user norm, and 16 sketch values) to a
predicted log-rank.  It stands in for the paper's rank table plus linear
interpolation (Sec. 4.1 and query step 3 of Sec. 4.3): both turn a user's
score for q into an estimate of r(q,u,P).  The network is

    a1 = W1 x + b1,  h1 = relu(a1)          (64)
    a2 = W2 h1 + b2, h2 = relu(a2)          (64)
    y  = w3 . h2 + b3                       (1)

and is trained on the mean squared error against z = ln r:

    L = (1/N) sum_i (y_i - z_i)^2

with Adam (Kingma & Ba, 2015: bias-corrected first and second moments).
Parameters are held as a dict of float64 arrays: W1 [64,18], b1 [64],
W2 [64,64], b2 [64], w3 [64], b3 [1].  relu'(0) is taken as 0.
"""
from __future__ import annotations

import numpy as np

SHAPES = {"W1": (64, 18), "b1": (64,), "W2": (64, 64), "b2": (64,), "w3": (64,), "b3": (1,)}
ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")


def n_params() -> int:
    return int(sum(np.prod(s) for s in SHAPES.values()))


def unflatten(flat) -> dict:
    flat = np.asarray(flat, np.float64)
    out, o = {}, 0
    for k in ORDER:
        sz = int(np.prod(SHAPES[k]))
        out[k] = flat[o:o + sz].reshape(SHAPES[k]).copy()
        o += sz
    assert o == flat.size
    return out


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], np.float64).ravel() for k in ORDER])


def forward(params: dict, X) -> tuple[np.ndarray, dict]:
    X = np.asarray(X, np.float64)
    a1 = X @ params["W1"].T + params["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ params["W2"].T + params["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ params["w3"] + params["b3"][0]
    return y, {"X": X, "a1": a1, "h1": h1, "a2": a2, "h2": h2}


def loss(params: dict, X, z) -> float:
    y, _ = forward(params, X)
    z = np.asarray(z, np.float64)
    return float(np.mean((y - z) ** 2))


def loss_and_grad(params: dict, X, z) -> tuple[float, dict]:
    y, c = forward(params, X)
    z = np.asarray(z, np.float64)
    N = y.shape[0]
    r = y - z
    L = float(np.mean(r * r))
    dy = 2.0 * r / N                       # dL/dy_i
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, params["w3"])
    da2 = dh2 * (c["a2"] > 0.0)
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ params["W2"]
    da1 = dh1 * (c["a1"] > 0.0)
    g["W1"] = da1.T @ c["X"]
    g["b1"] = da1.sum(axis=0)
    return L, g


def finite_difference(params: dict, X, z, h: float = 1e-6) -> np.ndarray:
    """Central differences of L over every parameter (flattened order)."""
    flat = flatten(params)
    out = np.empty_like(flat)
    for i in range(flat.size):
        fp = flat.copy(); fp[i] += h
        fm = flat.copy(); fm[i] -= h
        out[i] = (loss(unflatten(fp), X, z) - loss(unflatten(fm), X, z)) / (2.0 * h)
    return out


def adam_step(params: dict, grads: dict, m: dict, v: dict, t: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam update in place; t is the 1-based step count."""
    for k in ORDER:
        g = grads[k]
        m[k] = b1 * m[k] + (1.0 - b1) * g
        v[k] = b2 * v[k] + (1.0 - b2) * g * g
        mh = m[k] / (1.0 - b1 ** t)
        vh = v[k] / (1.0 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
