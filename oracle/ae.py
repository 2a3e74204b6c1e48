"""Autoencoder evaluation and training in FP64 (Section III Stages 2-3, Eq. 5; Section IV-C).

Dense model:  x = (f - mu) / sigma  (z-score per pixel, Section IV-D)
              z = W2 relu(W1 x + b1) + b2                       (encoder, linear latent)
              xhat = W4 relu(W3 z + b3) + b4,  fhat = sigma xhat + mu
Tied linear model (the paper's own, Section IV-C): z = W x,  xhat = W^T z.
Loss: MSE(X, Xhat), the mean over batch and pixels (Eq. 5).  Optimizer: Adam.
Weights are stored [out][in] (y = x @ W.T + b).
"""
from __future__ import annotations

import numpy as np


def relu(x):
    return np.maximum(x, 0.0)


def norm_stats(F: np.ndarray, floor_rel: float = 1e-12):
    """Per-pixel mean and population std over a batch (H, N); std floored at floor_rel*max std."""
    X = np.asarray(F, np.float64).reshape(F.shape[0], -1)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.maximum(sd, floor_rel * sd.max())
    return mu, sd


def _w(W, k):
    return np.asarray(W[k], np.float64)


def dense_encode(X: np.ndarray, W: dict) -> np.ndarray:
    """X: normalised inputs (B, N) -> latent (B, L)."""
    h1 = relu(X @ _w(W, "W1").T + _w(W, "b1"))
    return h1 @ _w(W, "W2").T + _w(W, "b2")


def dense_decode(Z: np.ndarray, W: dict) -> np.ndarray:
    """Latent (B, L) -> normalised reconstruction (B, N)."""
    h3 = relu(Z @ _w(W, "W3").T + _w(W, "b3"))
    return h3 @ _w(W, "W4").T + _w(W, "b4")


def normalize(F, mu, sd):
    return (np.asarray(F, np.float64).reshape(F.shape[0], -1) - mu) / sd


def denormalize(Xh, mu, sd):
    return sd * Xh + mu


def _mm(A, B, rnd):
    """A @ B in FP64; with rnd (the BF16 training form) both operands are rounded first."""
    if rnd is None:
        return A @ B
    return rnd(A).astype(np.float64) @ rnd(B).astype(np.float64)


def dense_forward_train(X: np.ndarray, W: dict, rnd=None):
    """Full forward pass with the values the backward pass needs.  rnd: None (FP64), or a
    rounding applied to both operands of every product (`bf16`: the BF16 training form,
    bfloat16 operands, exact products, FP32 master weights; biases and ReLU unrounded)."""
    a1 = _mm(X, _w(W, "W1").T, rnd) + _w(W, "b1")
    h1 = relu(a1)
    z = _mm(h1, _w(W, "W2").T, rnd) + _w(W, "b2")
    a3 = _mm(z, _w(W, "W3").T, rnd) + _w(W, "b3")
    h3 = relu(a3)
    xh = _mm(h3, _w(W, "W4").T, rnd) + _w(W, "b4")
    return dict(X=X, a1=a1, h1=h1, z=z, a3=a3, h3=h3, xh=xh)


def mse(xh: np.ndarray, X: np.ndarray) -> float:
    return float(np.mean((xh - X) ** 2))


def dense_backward(cache: dict, W: dict, rnd=None, dz_extra=None) -> dict:
    """Gradients of MSE(xhat, X) (mean over all B*N terms) w.r.t. every parameter, by the
    chain rule layer by layer; rnd as in `dense_forward_train` (both operands of every
    product of the backward pass rounded).  dz_extra: an extra dL/dz added at the latent."""
    X, h1, z, h3, xh = cache["X"], cache["h1"], cache["z"], cache["h3"], cache["xh"]
    B, N = X.shape
    dxh = 2.0 * (xh - X) / (B * N)
    g = {}
    g["W4"] = _mm(dxh.T, h3, rnd)
    g["b4"] = dxh.sum(axis=0)
    dh3 = _mm(dxh, _w(W, "W4"), rnd)
    da3 = dh3 * (cache["a3"] > 0)
    g["W3"] = _mm(da3.T, z, rnd)
    g["b3"] = da3.sum(axis=0)
    dz = _mm(da3, _w(W, "W3"), rnd)
    if dz_extra is not None:
        dz = dz + dz_extra
    g["W2"] = _mm(dz.T, h1, rnd)
    g["b2"] = dz.sum(axis=0)
    dh1 = _mm(dz, _w(W, "W2"), rnd)
    da1 = dh1 * (cache["a1"] > 0)
    g["W1"] = _mm(da1.T, X, rnd)
    g["b1"] = da1.sum(axis=0)
    return g


def dense_loss(X: np.ndarray, W: dict) -> float:
    return mse(dense_forward_train(X, W)["xh"], X)


def tied_forward(X: np.ndarray, Wt: np.ndarray):
    """The paper's tied linear AE: z = X W^T, xhat = z W (W is [L][N])."""
    z = X @ Wt.T
    return z, z @ Wt


def tied_grad(X: np.ndarray, Wt: np.ndarray) -> np.ndarray:
    z, xh = tied_forward(X, Wt)
    B, N = X.shape
    d = 2.0 * (xh - X) / (B * N)
    # xhat = X W^T W: dL/dW = z^T d + (d W^T)^T X
    return z.T @ d + (d @ Wt.T).T @ X


def adam_step(params: dict, grads: dict, state: dict, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) in place; `state` holds m, v and the step count t."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for k, gk in grads.items():
        m = state.setdefault("m_" + k, np.zeros_like(gk))
        v = state.setdefault("v_" + k, np.zeros_like(gk))
        m[...] = b1 * m + (1 - b1) * gk
        v[...] = b2 * v + (1 - b2) * gk * gk
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


# ---- BF16 form (matrix-core operands rounded to bfloat16, sums in higher precision) ----
#
# The dense model again, with the two large products taking bfloat16 operands: the
# encoder's input x and W1, the decoder's hidden h3 and W4.  Where a rounding to bfloat16
# decides a value, it is taken from the FP32 value the kernel forms (the rule for
# decisions made in floating point): x = (f - mu) * (1/sigma) in FP32, h3 by the FP32
# fused multiply-add chain b3 + sum_d zhat_d W3_cd in order d = 0..15.  The products of
# bfloat16 values are exact in FP64 and are summed there.

def bf16(x) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as FP32.
    Finite inputs only."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def fma32(a, b, c) -> np.ndarray:
    """FP32 fused multiply-add: a b + c rounded once to the nearest FP32 value (ties to
    even).  The product of two FP32 values is exact in FP64; the FP64 sum s and its
    rounding error e (Knuth's two-sum) hold a b + c exactly.  Rounding s to FP32 is right
    unless s sits exactly halfway between two FP32 values, where the sign of e decides."""
    p = np.float64(a) * np.float64(b)
    c = np.asarray(c, np.float64)
    s = p + c
    bb = s - p
    e = (p - (s - bb)) + (c - bb)
    r = s.astype(np.float32)
    other = np.nextafter(r, np.where(s > r, np.float32(np.inf), np.float32(-np.inf))).astype(np.float32)
    mid = (np.float64(r) != s) & ((np.float64(r) + np.float64(other)) * 0.5 == s)
    up = np.where(e > 0, np.maximum(r, other), np.minimum(r, other))
    return np.where(mid & (e != 0), up, r).astype(np.float32)


def bf16_encode_input(F32: np.ndarray, mu32: np.ndarray, rsd32: np.ndarray) -> np.ndarray:
    """x = (f - mu) * rsd in FP32 (non-finite inputs as 0), rounded to bfloat16."""
    f = np.where(np.isfinite(F32), F32, np.float32(0)).astype(np.float32)
    return bf16((f - mu32.astype(np.float32)) * rsd32.astype(np.float32))


def dense_encode_bf16(F32: np.ndarray, mu32, rsd32, W: dict) -> np.ndarray:
    """Latents of the BF16 form: h1 = relu(bf16(x) bf16(W1)^T + b1), z = h1 W2^T + b2."""
    H = F32.shape[0]
    xb = bf16_encode_input(F32.reshape(H, -1), mu32, rsd32).astype(np.float64)
    w1 = bf16(np.asarray(W["W1"], np.float32)).astype(np.float64)
    h1 = relu(xb @ w1.T + np.asarray(W["b1"], np.float64))
    return h1 @ np.asarray(W["W2"], np.float64).T + np.asarray(W["b2"], np.float64)


def dense_decode_bf16(Zh: np.ndarray, W: dict, mu, sd) -> np.ndarray:
    """fhat of the BF16 form: h3 by the FP32 FMA chain, rounded to bfloat16, then
    sigma (bf16(h3) bf16(W4)^T + b4) + mu."""
    W3 = np.asarray(W["W3"], np.float32)
    h3 = np.broadcast_to(np.asarray(W["b3"], np.float32), (Zh.shape[0], W3.shape[0])).astype(np.float32)
    Z32 = np.asarray(Zh, np.float32)
    for d in range(W3.shape[1]):
        h3 = fma32(Z32[:, d:d + 1], W3[None, :, d], h3)
    h3b = bf16(np.maximum(h3, np.float32(0))).astype(np.float64)
    w4 = bf16(np.asarray(W["W4"], np.float32)).astype(np.float64)
    y = h3b @ w4.T + np.asarray(W["b4"], np.float64)
    return np.asarray(sd, np.float64) * y + np.asarray(mu, np.float64)
