"""FP64 reference of the ordering MLP: forward, analytic backward, weighted BCE and Adam (numpy).

TEST INFRASTRUCTURE ONLY (gradient checks of the GPU kernels). The network scores a conditioning
candidate: 8 features -> 64 -> 64 -> 1 with ReLU. Parameters are one flat vector laid out as
W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3 (each weight row is one output unit).

Pinned in tests/test_oracle_mlp.py against torch.nn layers, torch autograd, torch's weighted
logit BCE and torch.optim.Adam (FP64, CPU), and against finite differences.
"""
from __future__ import annotations

import numpy as np

IN, HID = 8, 64
SIZES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def init(rng: np.random.Generator) -> np.ndarray:
    """He-style initialisation (weights N(0, 2/fan_in), biases 0)."""
    parts = []
    for name, shape in SIZES:
        if name.startswith("W"):
            fan_in = shape[-1] if len(shape) == 2 else HID
            parts.append(rng.standard_normal(int(np.prod(shape))) * np.sqrt(2.0 / fan_in))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts)


def forward(theta: np.ndarray, X: np.ndarray):
    p = unpack(np.asarray(theta, np.float64))
    X = np.asarray(X, np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    s = h2 @ p["W3"] + p["b3"][0]
    return s, (X, h1, h2)


def backward(theta: np.ndarray, cache, dscore: np.ndarray) -> np.ndarray:
    """Gradient of sum_r dscore[r] * score[r] with respect to theta (chain rule, layer by layer)."""
    p = unpack(np.asarray(theta, np.float64))
    X, h1, h2 = cache
    ds = np.asarray(dscore, np.float64)
    g = {"W3": h2.T @ ds, "b3": np.array([ds.sum()])}
    dz2 = np.outer(ds, p["W3"]) * (h2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * (h1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return np.concatenate([g[name].reshape(-1) for name, _ in SIZES])


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def bce(scores: np.ndarray, labels: np.ndarray, pos_weight: float):
    """Mean of w y softplus(-s) + (1 - y) softplus(s), and its derivative in s."""
    s = np.asarray(scores, np.float64)
    y = np.asarray(labels, np.float64)
    loss = np.mean(pos_weight * y * softplus(-s) + (1 - y) * softplus(s))
    sig = 1.0 / (1.0 + np.exp(-s))
    ds = (pos_weight * y * (sig - 1.0) + (1 - y) * sig) / s.size
    return loss, ds


def adam(theta, grad, m1, m2, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * grad
    m2 = b2 * m2 + (1 - b2) * grad * grad
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m1, m2
