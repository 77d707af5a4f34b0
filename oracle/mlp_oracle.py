"""FP64 CPU oracle of the warm-start network -- TEST INFRASTRUCTURE ONLY.

A fully connected network with three hidden ReLU layers of width H and one
linear output, trained by mean squared error with Adam (Kingma & Ba 2015).
Parameters are one flat vector in the order W1 (F x H), b1 (H), W2 (H x H),
b2, W3 (H x H), b3, w4 (H), b4 (1), matrices row-major (input index first).
The network is not part of the paper: it supplies a starting point to the
Newton iterations of Sec. 3, whose converged mode does not depend on it.
"""
from __future__ import annotations

import numpy as np


def shapes(F: int, H: int):
    return [("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
            ("w4", (H,)), ("b4", (1,))]


def n_params(F: int, H: int) -> int:
    return int(sum(np.prod(s) for _, s in shapes(F, H)))


def unpack(theta: np.ndarray, F: int, H: int):
    out, o = {}, 0
    for name, s in shapes(F, H):
        k = int(np.prod(s))
        out[name] = theta[o:o + k].reshape(s)
        o += k
    return out


def forward(theta: np.ndarray, X: np.ndarray, H: int):
    """Network output and the activations (pre-ReLU z_l, post-ReLU h_l)."""
    P = unpack(np.asarray(theta, np.float64), X.shape[1], H)
    z1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ P["W3"] + P["b3"]
    h3 = np.maximum(z3, 0.0)
    out = h3 @ P["w4"] + P["b4"][0]
    return out, (z1, h1, z2, h2, z3, h3)


def loss_and_grad(theta: np.ndarray, X: np.ndarray, target: np.ndarray, H: int):
    """L = mean_i (out_i - target_i)^2 and dL/dtheta by the chain rule."""
    n, F = X.shape
    P = unpack(np.asarray(theta, np.float64), F, H)
    out, (z1, h1, z2, h2, z3, h3) = forward(theta, X, H)
    r = out - target
    loss = float(np.mean(r * r))
    d_out = 2.0 * r / n
    g = {"w4": h3.T @ d_out, "b4": np.array([d_out.sum()])}
    d3 = np.outer(d_out, P["w4"]) * (z3 > 0)
    g["W3"], g["b3"] = h2.T @ d3, d3.sum(0)
    d2 = (d3 @ P["W3"].T) * (z2 > 0)
    g["W2"], g["b2"] = h1.T @ d2, d2.sum(0)
    d1 = (d2 @ P["W2"].T) * (z1 > 0)
    g["W1"], g["b1"] = X.T @ d1, d1.sum(0)
    flat = np.concatenate([g[name].ravel() for name, _ in shapes(F, H)])
    return loss, flat


def adam_step(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments), returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(F: int, H: int, rng: np.random.Generator) -> np.ndarray:
    """He-normal weights, zero biases."""
    parts = []
    for name, s in shapes(F, H):
        if name.startswith("W"):
            parts.append(rng.standard_normal(s).ravel() * np.sqrt(2.0 / s[0]))
        elif name == "w4":
            parts.append(rng.standard_normal(s) * np.sqrt(1.0 / s[0]))
        else:
            parts.append(np.zeros(int(np.prod(s))))
    return np.concatenate(parts)
