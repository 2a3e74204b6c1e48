"""Training of the dense autoencoder with the library's own kernels (Section III Stage 2,
Eq. 5; Sections IV-C and IV-D: Adam, z-scored inputs, a random sampler).

`DenseAE.apply(x, params)` is a torch.autograd.Function whose forward and backward are
hcz_ae_forward / hcz_ae_backward; `mse` wraps hcz_mse; `Trainer` runs Adam
(hcz_adam_step) over a device-resident training set.  torch provides memory, the random
permutation of the sampler and the autograd bookkeeping only.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import hcz
from .hcz import LIB, _check, _ptr, _stream

KEYS = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


def param_count(N: int) -> int:
    n = C.c_int64()
    _check(LIB.hcz_ae_param_count(N, C.byref(n)))
    return n.value


def shapes(N: int, hidden=hcz.HIDDEN, latent=hcz.LATENT):
    return dict(W1=(hidden, N), b1=(hidden,), W2=(latent, hidden), b2=(latent,), W3=(hidden, latent),
                b3=(hidden,), W4=(N, hidden), b4=(N,))


def pack(W: dict, device="cuda") -> torch.Tensor:
    return torch.from_numpy(hcz.pack_dense_weights(W)).to(device)


def unpack(p: torch.Tensor, N: int) -> dict:
    out, o = {}, 0
    flat = p.detach().cpu().numpy()
    for k, s in shapes(N).items():
        n = int(np.prod(s))
        out[k] = flat[o:o + n].reshape(s).copy()
        o += n
    return out


class DenseAE(torch.autograd.Function):
    """apply(x, params, compute=hcz.COMPUTE_FP32): with hcz.COMPUTE_BF16 every product of the
    forward and backward pass takes bfloat16 operands (FP32 accumulation and master weights)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, params: torch.Tensor, compute: int = hcz.COMPUTE_FP32):
        x = x.contiguous()
        B, N = x.shape
        nbytes = C.c_size_t()
        _check(LIB.hcz_ae_saved_bytes(N, B, C.byref(nbytes)))
        saved = torch.empty(max(nbytes.value, 4) // 4, dtype=torch.float32, device=x.device)
        z = torch.empty((B, hcz.LATENT), dtype=torch.float32, device=x.device)
        xh = torch.empty((B, N), dtype=torch.float32, device=x.device)
        _check(LIB.hcz_ae_forward(N, compute, _ptr(params), _ptr(x), B, _ptr(z), _ptr(xh), _ptr(saved),
                                  saved.numel() * 4, _stream()))
        ctx.save_for_backward(x, params, saved)
        ctx.compute = compute
        return z, xh

    @staticmethod
    def backward(ctx, dz, dxh):
        x, params, saved = ctx.saved_tensors
        B, N = x.shape
        grad = torch.empty_like(params)
        dx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        dz = None if dz is None else dz.contiguous()
        if dxh is None:
            dxh = torch.zeros_like(x)
        _check(LIB.hcz_ae_backward(N, ctx.compute, _ptr(params), _ptr(x), B, _ptr(dz), _ptr(dxh.contiguous()),
                                   _ptr(saved), saved.numel() * 4, _ptr(grad), _ptr(dx), _stream()))
        return dx, grad, None


def pack_conv(W: dict, device="cuda") -> torch.Tensor:
    """The convolutional model's parameters in the hcz_model_desc order (hcz.CONV_KEYS)."""
    return torch.from_numpy(np.concatenate([np.ascontiguousarray(W[k], np.float32).ravel()
                                            for k in hcz.CONV_KEYS])).to(device)


def unpack_conv(p: torch.Tensor) -> dict:
    from .synth import CONV_SHAPES
    out, o = {}, 0
    flat = p.detach().cpu().numpy()
    for k in hcz.CONV_KEYS:
        s = CONV_SHAPES[k]
        n = int(np.prod(s))
        out[k] = flat[o:o + n].reshape(s).copy()
        o += n
    return out


class ConvAE(torch.autograd.Function):
    """The convolutional model (39 x 39): hcz_conv_ae_forward / backward.  apply(x, params,
    compute=hcz.COMPUTE_FP32); with hcz.COMPUTE_BF16 every product of both passes takes
    bfloat16 operands (FP32 accumulation and master weights)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, params: torch.Tensor, compute: int = hcz.COMPUTE_FP32):
        x = x.contiguous()
        B = x.shape[0]
        nbytes = C.c_size_t()
        _check(LIB.hcz_conv_ae_saved_bytes(B, C.byref(nbytes)))
        saved = torch.empty(max(nbytes.value, 4) // 4, dtype=torch.float32, device=x.device)
        z = torch.empty((B, hcz.LATENT), dtype=torch.float32, device=x.device)
        xh = torch.empty((B, 1521), dtype=torch.float32, device=x.device)
        _check(LIB.hcz_conv_ae_forward(compute, _ptr(params), _ptr(x), B, _ptr(z), _ptr(xh), _ptr(saved),
                                       saved.numel() * 4, _stream()))
        ctx.save_for_backward(x, params, saved)
        ctx.compute = compute
        return z, xh

    @staticmethod
    def backward(ctx, dz, dxh):
        x, params, saved = ctx.saved_tensors
        B = x.shape[0]
        grad = torch.empty_like(params)
        dz = None if dz is None else dz.contiguous()
        if dxh is None:
            dxh = torch.zeros_like(x)
        _check(LIB.hcz_conv_ae_backward(ctx.compute, _ptr(params), _ptr(x), B, _ptr(dz), _ptr(dxh.contiguous()),
                                        _ptr(saved), saved.numel() * 4, _ptr(grad), _stream()))
        return None, grad, None


class MSE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xh: torch.Tensor, x: torch.Tensor):
        nbytes = C.c_size_t()
        _check(LIB.hcz_mse_workspace(C.byref(nbytes)))
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=x.device)
        loss = torch.empty((), dtype=torch.float32, device=x.device)
        dxh = torch.empty_like(xh)
        _check(LIB.hcz_mse(_ptr(xh.contiguous()), _ptr(x.contiguous()), xh.numel(), _ptr(loss), _ptr(dxh),
                           _ptr(ws), ws.numel(), _stream()))
        ctx.save_for_backward(dxh)
        return loss

    @staticmethod
    def backward(ctx, g):
        (dxh,) = ctx.saved_tensors
        return dxh * g, None


def mse(xh, x):
    return MSE.apply(xh, x)


class Trainer:
    """Adam on the packed parameter vector with hcz_adam_step (FP32 master weights)."""

    def __init__(self, params: torch.Tensor, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, arch: str = "dense",
                 compute: str = "fp32"):
        """compute: "fp32", or "bf16": bfloat16 operands in every product, FP32 accumulation,
        FP32 master weights and Adam state (dense and convolutional models)."""
        if compute not in ("fp32", "bf16") or arch not in ("dense", "conv"):
            raise ValueError("compute must be 'fp32' or 'bf16', arch 'dense' or 'conv'")
        self.arch = arch
        self.compute = hcz.COMPUTE_BF16 if compute == "bf16" else hcz.COMPUTE_FP32
        self.p = params.detach().clone().contiguous()
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.lr, self.betas, self.eps = lr, betas, eps
        self.step_count = 0

    def step(self, grad: torch.Tensor) -> None:
        self.step_count += 1
        _check(LIB.hcz_adam_step(_ptr(self.p), _ptr(grad.contiguous()), _ptr(self.m), _ptr(self.v),
                                 self.p.numel(), self.lr, self.betas[0], self.betas[1], self.eps,
                                 self.step_count, _stream()))

    def train_step(self, xb: torch.Tensor) -> torch.Tensor:
        p = self.p.detach().requires_grad_(True)
        _, xh = ConvAE.apply(xb, p, self.compute) if self.arch == "conv" else DenseAE.apply(xb, p, self.compute)
        loss = mse(xh, xb)
        loss.backward()
        self.step(p.grad)
        return loss.detach()

    def fit(self, X: torch.Tensor, epochs: int, batch: int = 1024, seed: int = 0, log=None) -> list:
        """X: z-scored training set [n][N] on the device; random sampler without replacement."""
        g = torch.Generator(device=X.device)
        g.manual_seed(seed)
        losses = []
        n = X.shape[0]
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g, device=X.device)
            tot = torch.zeros((), dtype=torch.float64, device=X.device)
            nb = 0
            for s in range(0, n - batch + 1, batch):
                tot += self.train_step(X[perm[s:s + batch]])
                nb += 1
            losses.append((tot / max(nb, 1)).item())
            if log:
                log(f"epoch {ep + 1}: loss {losses[-1]:.5f}")
        return losses


# ---- data selection and incremental training (Section IV-D) --------------------------------

def colrandind(planes: int, nodes: int, seed: int = 0) -> np.ndarray:
    """Training rows chosen like the paper's column-random-index scheme (Section IV-D,
    Fig. 5): the batch holds planes x nodes histograms (row r * nodes + m); for every mesh
    node m one plane r_m is drawn uniformly, giving `nodes` rows, one per node, in node
    order.  The draw is NumPy PCG64 with the given seed."""
    if planes < 1 or nodes < 0:
        raise ValueError("planes >= 1 and nodes >= 0")
    r = np.random.Generator(np.random.PCG64(seed)).integers(0, planes, size=nodes)
    return r.astype(np.int64) * nodes + np.arange(nodes, dtype=np.int64)


def incremental(params: torch.Tensor, X: torch.Tensor, epochs: int = 2, batch: int = 1024, lr: float = 1e-3,
                seed: int = 0, compute: str = "fp32") -> tuple:
    """Incremental training (Section IV-D): continue a model trained on an earlier batch
    with `epochs` passes over the current batch's z-scored rows X, with fresh Adam moments.
    Returns (Trainer, per-epoch losses)."""
    tr = Trainer(params, lr=lr, compute=compute)
    return tr, tr.fit(X, epochs=epochs, batch=batch, seed=seed)


# ---- warm-start network -------------------------------------------------------------------

MLP_KEYS = ("W1", "b1", "W2", "b2", "W3", "b3")
MLP_SHAPES = dict(W1=(64, 16), b1=(64,), W2=(64, 64), b2=(64,), W3=(4, 64), b3=(4,))


def mlp_pack(P: dict, device="cuda") -> torch.Tensor:
    return torch.from_numpy(np.concatenate([np.ascontiguousarray(P[k], np.float32).ravel()
                                            for k in MLP_KEYS])).to(device)


def mlp_unpack(p: torch.Tensor) -> dict:
    out, o = {}, 0
    flat = p.detach().cpu().numpy()
    for k in MLP_KEYS:
        n = int(np.prod(MLP_SHAPES[k]))
        out[k] = flat[o:o + n].reshape(MLP_SHAPES[k]).copy()
        o += n
    return out


class MlpNet(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z: torch.Tensor, params: torch.Tensor):
        z = z.contiguous()
        B = z.shape[0]
        nbytes = C.c_size_t()
        _check(LIB.hcz_mlp_saved_bytes(B, C.byref(nbytes)))
        saved = torch.empty(max(nbytes.value, 4) // 4, dtype=torch.float32, device=z.device)
        out = torch.empty((B, 4), dtype=torch.float32, device=z.device)
        _check(LIB.hcz_mlp_forward(_ptr(params), _ptr(z), B, _ptr(out), _ptr(saved), saved.numel() * 4, _stream()))
        ctx.save_for_backward(z, params, saved)
        return out

    @staticmethod
    def backward(ctx, dout):
        z, params, saved = ctx.saved_tensors
        grad = torch.empty_like(params)
        _check(LIB.hcz_mlp_backward(_ptr(params), _ptr(z), z.shape[0], _ptr(dout.contiguous()), _ptr(saved),
                                    saved.numel() * 4, _ptr(grad), _stream()))
        return None, grad


def fit_mlp(Z: torch.Tensor, T: torch.Tensor, P0: dict, epochs: int = 30, batch: int = 1024, lr: float = 1e-3,
            seed: int = 0) -> tuple[torch.Tensor, list]:
    """Train the warm-start network on latents Z [n][16] and scaled targets T [n][4] with MSE
    and Adam (hcz_adam_step); returns (packed parameters, per-epoch losses)."""
    tr = Trainer(mlp_pack(P0, Z.device), lr=lr)
    g = torch.Generator(device=Z.device)
    g.manual_seed(seed)
    losses = []
    n = Z.shape[0]
    for _ in range(epochs):
        perm = torch.randperm(n, generator=g, device=Z.device)
        tot, nb = torch.zeros((), dtype=torch.float64, device=Z.device), 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            p = tr.p.detach().requires_grad_(True)
            loss = mse(MlpNet.apply(Z[idx], p), T[idx].contiguous())
            loss.backward()
            tr.step(p.grad)
            tot += loss.detach()
            nb += 1
        losses.append((tot / max(nb, 1)).item())
    return tr.p, losses
