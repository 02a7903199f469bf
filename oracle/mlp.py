"""fp64 oracle of the learned cardinality estimator -- TEST INFRASTRUCTURE ONLY.

The paper has no learned part; this network is an addition of this project.  It maps the
per-age live-cell counts of a host's union SLE (x_a for ages a < 10) to the natural log of
the host's cardinality.  Each count is encoded as the log of that age's own linear-counting
estimate (Eq. 9 with eta' + 1 in the denominator so a full SLE stays finite), scaled by 1/8:

    phi_a = log1p(-eta' * log1p(-x_a / (eta' + 1))) / 8
    h1 = relu(W1 phi + b1)    W1: 64 x 10
    h2 = relu(W2 h1 + b2)     W2: 64 x 64
    y  = W3 h2 + b3           W3: 1 x 64
    loss = mean over the batch of (y - log c)^2

Adam (Kingma & Ba, 2015) updates the parameters.  Everything here is float64 numpy, written
from the definitions above so gradients can also be checked by finite differences.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 10, 64
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (1, N_H)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def init_params(seed: int) -> dict:
    """He-normal weights, zero biases."""
    rng = np.random.Generator(np.random.Philox(seed))
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            p[name] = rng.standard_normal(shape) * np.sqrt(2.0 / shape[1])
        else:
            p[name] = np.zeros(shape)
    return p


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[n], dtype=np.float64).ravel() for n, _ in SHAPES])


def unflatten(v: np.ndarray) -> dict:
    p, o = {}, 0
    for n, s in SHAPES:
        m = int(np.prod(s))
        p[n] = np.asarray(v[o:o + m], dtype=np.float64).reshape(s)
        o += m
    return p


def encode(x: np.ndarray, etap: int) -> np.ndarray:
    """Input encoding of per-age counts (fp64)."""
    x = np.asarray(x, dtype=np.float64)
    return np.log1p(-etap * np.log1p(-x / (etap + 1.0))) / 8.0


def forward(p: dict, x: np.ndarray):
    """x: (B, 10) encoded inputs.  Returns (y (B,), cache)."""
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ p["W3"].T + p["b3"])[:, 0]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(p: dict, x: np.ndarray, t: np.ndarray):
    """Mean squared error against targets t (log cardinality) and its analytic gradient."""
    y, (x, z1, h1, z2, h2) = forward(p, x)
    B = x.shape[0]
    d = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(d * d))
    dy = (2.0 / B) * d                        # (B,)
    g = {}
    g["W3"] = dy[None, :] @ h2                # (1, 64)
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] * p["W3"]               # (B, 64)
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(p: dict, g: dict, m: dict, v: dict, step: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    np_, nm, nv = {}, {}, {}
    for n, _ in SHAPES:
        nm[n] = b1 * m[n] + (1.0 - b1) * g[n]
        nv[n] = b2 * v[n] + (1.0 - b2) * g[n] * g[n]
        mh = nm[n] / (1.0 - b1 ** step)
        vh = nv[n] / (1.0 - b2 ** step)
        np_[n] = p[n] - lr * mh / (np.sqrt(vh) + eps)
    return np_, nm, nv
