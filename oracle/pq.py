"""Product quantisation of the latent vectors (Section III Stage 3; Section IV-E).

Each latent dimension d gets its own codebook of k = 2^bits sorted centroids, fitted by
1-D k-means on a sample of that column.  Reading of the unstated details:
  * initial centroids: the sorted sample at indices floor((2c+1) n / (2k)), c = 0..k-1;
  * Lloyd iterations until no assignment changes, at most 25 centroid updates;
  * a cluster with no members keeps its centroid;
  * the fit runs in FP64 and the centroids are stored FP32.
Encoding: code_d = #{c : beta_{d,c} < z_d} with midpoints beta_c = (C_c + C_{c+1}) * 0.5
in FP64 from the FP32 centroids; this selects the nearest centroid value, an exact
midpoint going to the lower one.
A vector of L dims then costs L * bits bits (Section III Stage 3) and the table
L * k * 4 bytes (Section IV-E).
"""
from __future__ import annotations

import numpy as np


def midpoints(C: np.ndarray) -> np.ndarray:
    C = np.asarray(C, np.float64)
    return (C[..., :-1] + C[..., 1:]) * 0.5


def assign_1d(z: np.ndarray, C: np.ndarray) -> np.ndarray:
    """#{c : beta_c < z} for every z (C sorted, so the midpoints are sorted and a left
    binary search returns exactly that count)."""
    beta = midpoints(C)
    z = np.asarray(z, np.float64)
    a = np.searchsorted(beta, z, side="left")
    a[np.isnan(z)] = 0            # no midpoint is below NaN
    return a


def fit_1d(sample: np.ndarray, k: int, max_iter: int = 25):
    """Lloyd's algorithm in 1-D; returns (FP64 centroids, number of updates)."""
    s = np.sort(np.asarray(sample, np.float64))
    n = s.size
    C = s[((2 * np.arange(k) + 1) * n) // (2 * k)].copy()
    prev = None
    updates = 0
    for _ in range(max_iter):
        a = assign_1d(s, C)
        if prev is not None and np.array_equal(a, prev):
            break
        for c in np.unique(a):
            C[c] = s[a == c].mean()
        prev = a
        updates += 1
    return C, updates


def fit(Z: np.ndarray, bits: int = 8, sample_every: int = 1, max_iter: int = 25) -> np.ndarray:
    """Codebook (L, 2^bits) FP32 from the rows Z[::sample_every] of a latent matrix (n, L)."""
    S = np.asarray(Z)[::sample_every]
    k = 1 << bits
    return np.stack([fit_1d(S[:, d], k, max_iter)[0] for d in range(S.shape[1])]).astype(np.float32)


def encode(Z: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Codes (n, L) uint8 for latents Z (n, L) under codebook C (L, k)."""
    Z = np.asarray(Z)
    out = np.empty(Z.shape, dtype=np.uint8)
    for d in range(Z.shape[1]):
        out[:, d] = assign_1d(Z[:, d].astype(np.float64), C[d])
    return out


def decode(codes: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Dequantised latents zhat[n, d] = C[d, code[n, d]] (FP64 view of the FP32 table)."""
    d = np.arange(codes.shape[1])[None, :]
    return np.asarray(C, np.float64)[d, codes.astype(np.int64)]


def kmeans_cost(s: np.ndarray, C: np.ndarray) -> float:
    s = np.asarray(s, np.float64)
    return float(np.min((s[:, None] - np.asarray(C, np.float64)[None, :]) ** 2, axis=1).sum())
