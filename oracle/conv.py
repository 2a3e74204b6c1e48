"""Convolutional autoencoder for 39 x 39 histograms in its BF16 form (Section III Stage 2,
the precision form of the autoencoder step): test infrastructure, FP64 NumPy.

Encoder:  x = (f - mu) * (1/sigma) in FP32 (non-finite inputs as 0), 39 x 39
          h1 = relu(conv1(x))       3x3, 1 -> 32, stride 2, padding 1 -> 20 x 20
          h2 = relu(conv2(h1))      3x3, 32 -> 64, stride 2, padding 1 -> 10 x 10
          z  = fw h2 + fb           6400 -> 16 (h2 flattened channel-major), linear
Decoder:  hd = relu(dw zhat + db)   16 -> 6400, viewed as 64 x 10 x 10
          h3 = relu(convT1(hd))     transposed 3x3, 64 -> 32, stride 2, padding 1,
                                    output padding 1 -> 20 x 20
          y  = convT2(h3)           transposed 3x3, 32 -> 1, stride 2, padding 1 -> 39 x 39
          fhat = sigma y + mu
The plain FP64 model (encode64 / decode64) evaluates the same layers in FP64 throughout;
it is the reference the BF16 form's error is stated against.
BF16 form: the operands of conv2 and convT1 (h1, hd and their weights) are rounded to
nearest-even bfloat16.  Both rounded activations come from FP32 fused multiply-add chains
that the oracle reproduces exactly: h1 = b1 + sum over the window's in-range taps in
row-major order (ky, then kx) of x w; hd = db + sum over d = 0..15 of zhat_d dw[:, d].
Everything else is evaluated in FP64 (products of the FP32/bfloat16 values summed in
FP64).  A tap outside the input (padding) contributes nothing.
"""
from __future__ import annotations

import numpy as np

from .ae import bf16, bf16_encode_input, fma32, relu  # noqa: F401


def _x32(F32: np.ndarray, mu32, rsd32) -> np.ndarray:
    H = F32.shape[0]
    f = np.where(np.isfinite(F32), F32, np.float32(0)).astype(np.float32).reshape(H, 39, 39)
    return (f - np.asarray(mu32, np.float32).reshape(39, 39)) * np.asarray(rsd32, np.float32).reshape(39, 39)


def conv1_fp32(x32: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """relu(conv1(x)) as the FP32 chain described above: (H, 32, 20, 20) FP32."""
    H = x32.shape[0]
    w = np.asarray(w, np.float32)
    s = np.broadcast_to(np.asarray(b, np.float32)[None, :, None, None], (H, 32, 20, 20)).astype(np.float32)
    oy = np.arange(20)
    for ky in range(3):
        iy = 2 * oy - 1 + ky
        vy = (iy >= 0) & (iy < 39)
        for kx in range(3):
            ix = 2 * oy - 1 + kx
            vx = (ix >= 0) & (ix < 39)
            xv = x32[:, np.clip(iy, 0, 38)][:, :, np.clip(ix, 0, 38)]          # (H, 20, 20)
            t = fma32(xv[:, None], w[None, :, 0, ky, kx, None, None], s)
            s = np.where((vy[:, None] & vx[None, :])[None, None], t, s).astype(np.float32)
    return np.maximum(s, np.float32(0))


def conv2d_s2(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """3x3 convolution, stride 2, padding 1, FP64: x (H, C, n, n), w (O, C, 3, 3)."""
    H, C, n, _ = x.shape
    m = (n + 2 - 3) // 2 + 1
    xp = np.zeros((H, C, n + 2, n + 2))
    xp[:, :, 1:n + 1, 1:n + 1] = x
    out = np.zeros((H, w.shape[0], m, m))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + 2 * m - 1:2, kx:kx + 2 * m - 1:2]      # (H, C, m, m)
            out += np.einsum('hcij,oc->hoij', patch, np.asarray(w[:, :, ky, kx], np.float64), optimize=True)
    return out + np.asarray(b, np.float64)[None, :, None, None]


def conv_t2d_s2(x: np.ndarray, w: np.ndarray, b: np.ndarray, out_n: int) -> np.ndarray:
    """3x3 transposed convolution, stride 2, padding 1 (output padding so that the output
    is out_n x out_n), FP64: x (H, C, n, n), w (C, O, 3, 3).  Input cell (iy, ix) adds
    x w[., ., ky, kx] to output cell (2 iy - 1 + ky, 2 ix - 1 + kx)."""
    H, C, n, _ = x.shape
    O = w.shape[1]
    full = np.zeros((H, O, 2 * n + 1, 2 * n + 1))          # output index + 1
    for ky in range(3):
        for kx in range(3):
            full[:, :, ky:ky + 2 * n - 1:2, kx:kx + 2 * n - 1:2] += np.einsum(
                'hcij,co->hoij', x, np.asarray(w[:, :, ky, kx], np.float64), optimize=True)
    return full[:, :, 1:out_n + 1, 1:out_n + 1] + np.asarray(b, np.float64)[None, :, None, None]


def encode_bf16(F32: np.ndarray, mu32, rsd32, W: dict) -> np.ndarray:
    """Latents z (H, 16) of the BF16 form."""
    H = F32.shape[0]
    h1 = conv1_fp32(_x32(F32, mu32, rsd32), W["c1w"], W["c1b"])
    h2 = relu(conv2d_s2(bf16(h1).astype(np.float64), bf16(W["c2w"]).astype(np.float64), W["c2b"]))
    return h2.reshape(H, 6400) @ np.asarray(W["fw"], np.float64).T + np.asarray(W["fb"], np.float64)


def dec_hidden_fp32(Zh: np.ndarray, W: dict) -> np.ndarray:
    """relu(dw zhat + db) by the FP32 chain over d = 0..15: (H, 6400) FP32."""
    dw = np.asarray(W["dw"], np.float32)
    s = np.broadcast_to(np.asarray(W["db"], np.float32), (Zh.shape[0], 6400)).astype(np.float32)
    Z32 = np.asarray(Zh, np.float32)
    for d in range(16):
        s = fma32(Z32[:, d:d + 1], dw[None, :, d], s)
    return np.maximum(s, np.float32(0))


def decode_bf16(Zh: np.ndarray, W: dict, mu, sd) -> np.ndarray:
    """fhat (H, 1521) of the BF16 form."""
    H = Zh.shape[0]
    hd = bf16(dec_hidden_fp32(Zh, W)).astype(np.float64).reshape(H, 64, 10, 10)
    h3 = relu(conv_t2d_s2(hd, bf16(W["t1w"]).astype(np.float64), W["t1b"], 20))
    y = conv_t2d_s2(h3, np.asarray(W["t2w"], np.float64), W["t2b"], 39).reshape(H, 1521)
    return np.asarray(sd, np.float64) * y + np.asarray(mu, np.float64)


# ---- the plain FP64 model (no bfloat16, no FP32 chains) ----------------------------------

def encode64(F64: np.ndarray, mu, sd, W: dict) -> np.ndarray:
    """Latents z (H, 16) of the plain FP64 model: x = (f - mu) / sigma, then conv1, ReLU,
    conv2, ReLU and the dense layer, every value and product in FP64 with the stored
    weights widened exactly.  The reference the BF16 form's error is stated against."""
    H = F64.shape[0]
    x = ((np.asarray(F64, np.float64).reshape(H, 1521) - np.asarray(mu, np.float64))
         / np.asarray(sd, np.float64)).reshape(H, 1, 39, 39)
    w = {k: np.asarray(v, np.float64) for k, v in W.items()}
    h1 = relu(conv2d_s2(x, w["c1w"], w["c1b"]))
    h2 = relu(conv2d_s2(h1, w["c2w"], w["c2b"])).reshape(H, 6400)
    return h2 @ w["fw"].T + w["fb"]


def decode64(Zh: np.ndarray, W: dict, mu, sd) -> np.ndarray:
    """fhat (H, 1521) of the plain FP64 model from dequantised latents."""
    H = Zh.shape[0]
    w = {k: np.asarray(v, np.float64) for k, v in W.items()}
    hd = relu(np.asarray(Zh, np.float64) @ w["dw"].T + w["db"]).reshape(H, 64, 10, 10)
    h3 = relu(conv_t2d_s2(hd, w["t1w"], w["t1b"], 20))
    y = conv_t2d_s2(h3, w["t2w"], w["t2b"], 39).reshape(H, 1521)
    return np.asarray(sd, np.float64) * y + np.asarray(mu, np.float64)


# ---- training (FP64): MSE loss (Eq. 5); rnd = None is the FP64 model throughout, rnd = bf16
# the BF16 training form (both operands of every product rounded, products exact, sums in
# FP64 here; biases, ReLU and the bias gradients unrounded) ------------------------------

def _r(a, rnd):
    return a if rnd is None else rnd(a).astype(np.float64)


def forward_train(X: np.ndarray, W: dict, rnd=None) -> dict:
    """Forward pass on z-scored rows X (B, 1521), keeping what the backward pass needs."""
    B = X.shape[0]
    x = np.asarray(X, np.float64).reshape(B, 1, 39, 39)
    w = {k: np.asarray(v, np.float64) for k, v in W.items()}
    r = lambda a: _r(a, rnd)          # noqa: E731
    a1 = conv2d_s2(r(x), r(w["c1w"]), w["c1b"])
    h1 = relu(a1)
    a2 = conv2d_s2(r(h1), r(w["c2w"]), w["c2b"])
    h2 = relu(a2).reshape(B, 6400)
    z = r(h2) @ r(w["fw"]).T + w["fb"]
    a4 = r(z) @ r(w["dw"]).T + w["db"]
    h4 = relu(a4).reshape(B, 64, 10, 10)
    a5 = conv_t2d_s2(r(h4), r(w["t1w"]), w["t1b"], 20)
    h5 = relu(a5)
    xh = conv_t2d_s2(r(h5), r(w["t2w"]), w["t2b"], 39).reshape(B, 1521)
    return dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, z=z, a4=a4, h4=h4, a5=a5, h5=h5, xh=xh)


def _wgrad(coarse: np.ndarray, fine: np.ndarray) -> np.ndarray:
    """G[cc, cf, ky, kx] = sum_b sum_(p) coarse[b, cc, py, px] fine[b, cf, 2py-1+ky, 2px-1+kx]
    (zero outside the fine grid): the weight gradient of a stride-2, padding-1 layer."""
    B, Cc, m, _ = coarse.shape
    Cf, n = fine.shape[1], fine.shape[2]
    fp = np.zeros((B, Cf, max(n + 2, 2 * m + 1), max(n + 2, 2 * m + 1)))
    fp[:, :, 1:n + 1, 1:n + 1] = fine
    G = np.zeros((Cc, Cf, 3, 3))
    for ky in range(3):
        for kx in range(3):
            patch = fp[:, :, ky:ky + 2 * m - 1:2, kx:kx + 2 * m - 1:2]
            G[:, :, ky, kx] = np.einsum('bcij,bfij->cf', coarse, patch, optimize=True)
    return G


def backward(cache: dict, W: dict, dxh: np.ndarray, dz: np.ndarray | None = None, rnd=None) -> dict:
    """Gradients of every parameter for dL/dxhat = dxh (B, 1521) (plus dL/dz = dz); rnd as in
    `forward_train` (both operands of every product of the backward pass rounded)."""
    B = dxh.shape[0]
    w = {k: np.asarray(v, np.float64) for k, v in W.items()}
    r = lambda a: _r(a, rnd)          # noqa: E731
    g = {}
    d = np.asarray(dxh, np.float64).reshape(B, 1, 39, 39)
    g["t2w"] = _wgrad(r(cache["h5"]), r(d))
    g["t2b"] = d.sum(axis=(0, 2, 3))
    d5 = conv2d_s2(r(d), r(w["t2w"]), np.zeros(32)) * (cache["a5"] > 0)
    g["t1w"] = _wgrad(r(cache["h4"]), r(d5))
    g["t1b"] = d5.sum(axis=(0, 2, 3))
    d4 = conv2d_s2(r(d5), r(w["t1w"]), np.zeros(64)).reshape(B, 6400) * (cache["a4"] > 0)
    g["dw"] = r(d4).T @ r(cache["z"])
    g["db"] = d4.sum(axis=0)
    dzt = r(d4) @ r(w["dw"]) + (0.0 if dz is None else np.asarray(dz, np.float64))
    g["fw"] = r(dzt).T @ r(cache["h2"])
    g["fb"] = dzt.sum(axis=0)
    d2 = (r(dzt) @ r(w["fw"])).reshape(B, 64, 10, 10) * (cache["a2"] > 0)
    g["c2w"] = _wgrad(r(d2), r(cache["h1"]))
    g["c2b"] = d2.sum(axis=(0, 2, 3))
    d1 = conv_t2d_s2(r(d2), r(w["c2w"]), np.zeros(32), 20) * (cache["a1"] > 0)
    g["c1w"] = _wgrad(r(d1), r(cache["x"]))
    g["c1b"] = d1.sum(axis=(0, 2, 3))
    return g


def loss(X: np.ndarray, W: dict) -> float:
    return float(np.mean((forward_train(X, W)["xh"] - np.asarray(X, np.float64)) ** 2))
