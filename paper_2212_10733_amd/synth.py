"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle's tests.

This module draws random numbers and arranges them into arrays; it holds none of the
compression method's arithmetic (no moments, no norms, no network evaluation, no coding).

Velocity-space histograms stand in for the XGC ITER F-data of Section IV-A (not
available here).  Each histogram is a sum of 1-3 axis-aligned Gaussian bumps on a
uniform (v_perp, v_par) grid plus additive noise, clipped at zero:

    K ~ U{1,2,3};  per bump: c_par ~ U[-2,2], c_perp ~ U[0,2],
    s_par, s_perp ~ U[0.3,1.2], w ~ U[0.2,1]
    f[j,i] = sum_c w_c * gx_c[i] * gy_c[j],  gx = exp(-((v_par-c_par)/s_par)^2/2), ...
    f <- max(0, f + 1e-3 * max(f) * eps),    eps ~ N(0,1) iid

Draw order: chunks of 65,536 histograms, each with its own PCG64 stream spawned from
SeedSequence(seed); within a chunk all bump parameters first, then the noise in
sub-blocks of 8,192 histograms in order.  Storage is [H][n_perp][n_par] (row = v_perp).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 65536
SUB = 8192

# Seeds of the named workloads.
SEED_WEIGHTS = 0
SEED_PLAIN_SMALL = 1      # 256 histograms, FP64
SEED_PLAIN_LARGE = 2      # 2^20 histograms, FP32 (also the precision form)
SEED_TRAIN = 3
SEED_HELDOUT = 4
SEED_BATCHED = 5
SEED_SERIES = 11          # drifting series for incremental training: seed SEED_SERIES + t


def _axis(lo: float, hi: float, n: int) -> np.ndarray:
    return lo + (hi - lo) * np.arange(n, dtype=np.float64) / (n - 1)


def histograms(H: int, n_par: int = 39, n_perp: int = 39, seed: int = SEED_PLAIN_SMALL,
               dtype=np.float32, vpar=(-4.0, 4.0), vperp=(0.0, 4.0),
               threads: int | None = None, out: np.ndarray | None = None,
               shift: tuple = (0.0, 0.0)) -> np.ndarray:
    """Return H synthetic histograms, shape (H, n_perp, n_par), in `dtype`.
    shift: (dpar, dperp) added to every bump centre after the draws (the same random
    numbers, so shift = (0, 0) is the unshifted batch): a drifting series of batches."""
    if out is None:
        out = np.empty((H, n_perp, n_par), dtype=dtype)
    xs = _axis(vpar[0], vpar[1], n_par)
    ys = _axis(vperp[0], vperp[1], n_perp)
    n_chunks = max(1, math.ceil(H / CHUNK))
    children = np.random.SeedSequence(seed).spawn(n_chunks)

    def work(c: int) -> None:
        lo = c * CHUNK
        n = min(CHUNK, H - lo)
        if n <= 0:
            return
        rng = np.random.Generator(np.random.PCG64(children[c]))
        K = rng.integers(1, 4, size=n)
        cpar = rng.uniform(-2.0, 2.0, size=(n, 3))
        cperp = rng.uniform(0.0, 2.0, size=(n, 3))
        cpar = cpar + shift[0]
        cperp = cperp + shift[1]
        spar = rng.uniform(0.3, 1.2, size=(n, 3))
        sperp = rng.uniform(0.3, 1.2, size=(n, 3))
        w = rng.uniform(0.2, 1.0, size=(n, 3))
        w = np.where(np.arange(3)[None, :] < K[:, None], w, 0.0)
        for s in range(0, n, SUB):
            e = min(n, s + SUB)
            gx = np.exp(-0.5 * ((xs[None, None, :] - cpar[s:e, :, None]) / spar[s:e, :, None]) ** 2)
            gy = np.exp(-0.5 * ((ys[None, None, :] - cperp[s:e, :, None]) / sperp[s:e, :, None]) ** 2)
            f = np.einsum('nc,ncj,nci->nji', w[s:e], gy, gx, optimize=True)
            eps = rng.standard_normal(size=(e - s, n_perp, n_par))
            fmax = f.reshape(e - s, -1).max(axis=1)
            f += (1e-3 * fmax)[:, None, None] * eps
            np.maximum(f, 0.0, out=f)
            out[lo + s:lo + e] = f.astype(dtype)

    nthreads = threads or min(8, os.cpu_count() or 1)
    if n_chunks == 1 or nthreads == 1:
        for c in range(n_chunks):
            work(c)
    else:
        with ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(work, range(n_chunks)))
    return out


def xavier(fan_out: int, fan_in: int, rng: np.random.Generator) -> np.ndarray:
    a = math.sqrt(6.0 / (fan_in + fan_out))
    return rng.uniform(-a, a, size=(fan_out, fan_in)).astype(np.float32)


def dense_ae_weights(N: int = 1521, hidden: int = 128, latent: int = 16,
                     seed: int = SEED_WEIGHTS) -> dict:
    """Xavier-uniform weights of the dense autoencoder N->hidden->latent->hidden->N.

    Layout follows y = x @ W.T + b (W is [out][in]).  Biases are zero.  Draw order:
    W1, W2, W3, W4 from one PCG64 stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = xavier(hidden, N, rng)
    W2 = xavier(latent, hidden, rng)
    W3 = xavier(hidden, latent, rng)
    W4 = xavier(N, hidden, rng)
    z = lambda n: np.zeros(n, np.float32)
    return dict(W1=W1, b1=z(hidden), W2=W2, b2=z(latent), W3=W3, b3=z(hidden), W4=W4, b4=z(N))


def mlp_weights(sizes=(16, 64, 64, 4), seed: int = 6) -> dict:
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {}
    for li in range(len(sizes) - 1):
        out[f"W{li + 1}"] = xavier(sizes[li + 1], sizes[li], rng)
        out[f"b{li + 1}"] = np.zeros(sizes[li + 1], np.float32)
    return out


def latents(n: int, L: int = 16, seed: int = 7, dtype=np.float32) -> np.ndarray:
    """Latent-like samples: per dim a 3-component Gaussian mixture, shape (n, L)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.normal(0.0, 2.0, size=(L, 3))
    widths = rng.uniform(0.2, 1.0, size=(L, 3))
    comp = rng.integers(0, 3, size=(n, L))
    eps = rng.standard_normal(size=(n, L))
    d = np.arange(L)[None, :]
    return (centres[d, comp] + widths[d, comp] * eps).astype(dtype)


def sorted_codebook(L: int = 16, bits: int = 8, seed: int = 8) -> np.ndarray:
    """Random sorted FP32 centroids, shape (L, 2**bits)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    C = np.sort(rng.normal(0.0, 2.0, size=(L, 1 << bits)), axis=1)
    return C.astype(np.float32)


def perturbed(f: np.ndarray, rel: np.ndarray | float, seed: int = 9,
              dtype=np.float32) -> np.ndarray:
    """A stand-in reconstruction: f + rel * max(f) * eps per histogram (eps ~ N(0,1))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = f.shape[0]
    rel = np.broadcast_to(np.asarray(rel, np.float64), (H,))
    fmax = f.reshape(H, -1).max(axis=1).astype(np.float64)
    eps = rng.standard_normal(size=f.shape)
    return (f.astype(np.float64) + (rel * fmax)[:, None, None] * eps).astype(dtype)


def codes(n: int, L: int = 16, bits: int = 8, seed: int = 10) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 1 << bits, size=(n, L), dtype=np.uint8)


def series_shift(t: int) -> tuple:
    """Drift of the bump centres at step t of the synthetic series (velocity units)."""
    return (0.15 * t, 0.05 * t)


def series(t: int, planes: int, nodes: int, n_par: int = 39, n_perp: int = 39, dtype=np.float32) -> np.ndarray:
    """Step t of a drifting series: planes x nodes histograms, histogram (r, m) at row
    r * nodes + m (r: plane, m: mesh node), bump centres moved by series_shift(t)."""
    return histograms(planes * nodes, n_par, n_perp, seed=SEED_SERIES + t, dtype=dtype,
                      shift=series_shift(t))


BATCH_GRIDS = (33, 39, 49, 65)


def subdomains(n: int = 512, seed: int = SEED_BATCHED, count_range=(500, 20000), tau_range=(1e-4, 1e-2),
               grids=BATCH_GRIDS) -> list:
    """Layout of a batch of uneven subdomains: for each, (grid size g of a g x g grid,
    histogram count, tau), counts and tau log-uniform over their ranges, grids uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.integers(0, len(grids), size=n)
    c = np.exp(rng.uniform(math.log(count_range[0]), math.log(count_range[1]), size=n)).astype(np.int64)
    t = np.exp(rng.uniform(math.log(tau_range[0]), math.log(tau_range[1]), size=n))
    return [(int(grids[g[i]]), int(c[i]), float(t[i])) for i in range(n)]


CONV_SHAPES = dict(c1w=(32, 1, 3, 3), c1b=(32,), c2w=(64, 32, 3, 3), c2b=(64,), fw=(16, 6400), fb=(16,),
                   dw=(6400, 16), db=(6400,), t1w=(64, 32, 3, 3), t1b=(32,), t2w=(32, 1, 3, 3), t2b=(1,))
CONV_KEYS = tuple(CONV_SHAPES)


def conv_ae_weights(seed: int = SEED_WEIGHTS) -> dict:
    """Xavier-uniform weights of the convolutional autoencoder for 39 x 39 grids:
    conv 3x3 1->32 and 32->64 (stride 2, padding 1: 39 -> 20 -> 10), dense 6400 -> 16;
    decoder dense 16 -> 6400, transposed conv 64 -> 32 (stride 2, padding 1, output
    padding 1: 10 -> 20) and 32 -> 1 (stride 2, padding 1: 20 -> 39).  Shapes as in
    CONV_SHAPES (conv weights [out][in][ky][kx], transposed conv [in][out][ky][kx], dense
    [out][in]); fan sizes count the 3 x 3 window.  Biases are zero.  Draw order: c1w, c2w,
    fw, dw, t1w, t2w from one PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {}
    for k, s in CONV_SHAPES.items():
        if len(s) == 1:
            out[k] = np.zeros(s, np.float32)
            continue
        rf = s[2] * s[3] if len(s) == 4 else 1
        fan_sum = (s[0] + s[1]) * rf
        a = math.sqrt(6.0 / fan_sum)
        out[k] = rng.uniform(-a, a, size=s).astype(np.float32)
    return out
