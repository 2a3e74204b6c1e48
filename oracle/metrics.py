"""Error and size metrics (Eq. 7 and Section IV-A).

NRMSE(u, f) = sqrt(sum (u - f)^2 / N) / (max u - min u); the compression ratio is the
original size over the compressed size.
"""
from __future__ import annotations

import math

import numpy as np


def nrmse(u: np.ndarray, f: np.ndarray) -> float:
    u = np.asarray(u, np.float64).ravel()
    f = np.asarray(f, np.float64).ravel()
    return math.sqrt(math.fsum((u - f) ** 2) / u.size) / (u.max() - u.min())


def compressed_bytes(H: int, latent: int, bits: int, stream_bytes: int, lam_bytes: int = 8,
                     model_bytes: int = 0, codebook_bytes: int = 0, header: int = 44) -> int:
    """Codes (latent*bits bits per histogram), 4 multipliers, one flag byte per histogram,
    the residual stream, plus the model, codebook and a 44-byte header (Section III)."""
    return (H * latent * bits + 7) // 8 + H * 4 * lam_bytes + H + stream_bytes + model_bytes \
        + codebook_bytes + header


def compression_ratio(original_bytes: int, compressed: int) -> float:
    return original_bytes / compressed
