"""Warm-start multiplier network (the learned addition to Section III Stage 5).

A 16 -> 64 -> 64 -> 4 ReLU network maps the dequantised latent of a histogram to a first
guess of its four multipliers, in units of a per-component scale stored with the network:
lam0 = scale * (W3 relu(W2 relu(W1 zhat + b1) + b2) + b3).  Trained by MSE against the
multipliers the cold-start Newton solve produces (targets divided by the scale).
Cold start stays the fallback and the reference result (see newton.project).
"""
from __future__ import annotations

import numpy as np

from .ae import relu


def forward(Z: np.ndarray, P: dict):
    Z = np.asarray(Z, np.float64)
    a1 = Z @ np.asarray(P["W1"], np.float64).T + P["b1"]
    h1 = relu(a1)
    a2 = h1 @ np.asarray(P["W2"], np.float64).T + P["b2"]
    h2 = relu(a2)
    out = h2 @ np.asarray(P["W3"], np.float64).T + P["b3"]
    return dict(Z=Z, a1=a1, h1=h1, a2=a2, h2=h2, out=out)


def predict(Z, P, scale):
    return forward(Z, P)["out"] * np.asarray(scale, np.float64)


def loss(Z, T, P) -> float:
    return float(np.mean((forward(Z, P)["out"] - T) ** 2))


def backward(cache: dict, T: np.ndarray, P: dict) -> dict:
    """Gradients of mean((out - T)^2) over all B*4 terms."""
    out = cache["out"]
    B = out.shape[0]
    d = 2.0 * (out - T) / out.size
    g = {"W3": d.T @ cache["h2"], "b3": d.sum(0)}
    dh2 = d @ np.asarray(P["W3"], np.float64)
    da2 = dh2 * (cache["a2"] > 0)
    g["W2"] = da2.T @ cache["h1"]
    g["b2"] = da2.sum(0)
    dh1 = da2 @ np.asarray(P["W2"], np.float64)
    da1 = dh1 * (cache["a1"] > 0)
    g["W1"] = da1.T @ cache["Z"]
    g["b1"] = da1.sum(0)
    return g
