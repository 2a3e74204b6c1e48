"""Moments and quantities of interest (Section II, Eq. 1-4).

b = A f with correctly rounded sums (math.fsum).  The QoIs follow from b:
    n = b0,  u_par = V_par b1 / b0,  T_perp = (m/2) V_perp^2 b2 / b0,
    T_par = (m/2) (V_par^2 b3 / b0 - u_par^2).
`qoi_direct` evaluates Eq. 1-4 literally (T_par two-pass, around u_par) for reporting.
"""
from __future__ import annotations

import math

import numpy as np

from .grid import Grid


def moments(f: np.ndarray, g: Grid) -> np.ndarray:
    """b for one histogram f (n_perp, n_par) or a batch (H, n_perp, n_par); FP64."""
    A = g.A()
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 2:
        x = f.reshape(-1)
        return np.array([math.fsum(A[k] * x) for k in range(4)])
    return np.stack([moments(fh, g) for fh in f])


def qoi_from_moments(b: np.ndarray, g: Grid) -> np.ndarray:
    """(..., 4) moments -> (..., 4) QoIs [n, u_par, T_perp, T_par]."""
    b = np.asarray(b, dtype=np.float64)
    n = b[..., 0]
    u = g.Vpar * b[..., 1] / n
    tperp = 0.5 * g.mass * g.Vperp ** 2 * b[..., 2] / n
    tpar = 0.5 * g.mass * (g.Vpar ** 2 * b[..., 3] / n - u * u)
    return np.stack([n, u, tperp, tpar], axis=-1)


def qoi(f: np.ndarray, g: Grid) -> np.ndarray:
    return qoi_from_moments(moments(f, g), g)


def qoi_direct(f: np.ndarray, g: Grid) -> np.ndarray:
    """Eq. 1-4 term by term for one histogram (T_par around u_par, two passes)."""
    f = np.asarray(f, dtype=np.float64)
    w = f * g.vol
    vpar = np.broadcast_to(g.vpar[None, :], f.shape)
    vperp = np.broadcast_to(g.vperp[:, None], f.shape)
    n = math.fsum(w.ravel())
    u = math.fsum((w * vpar).ravel()) / n
    tperp = 0.5 * math.fsum((w * g.mass * vperp ** 2).ravel()) / n
    tpar = 0.5 * math.fsum((w * g.mass * (vpar - u) ** 2).ravel()) / n
    return np.array([n, u, tperp, tpar])


def qoi_rel_error(q_ref: np.ndarray, q: np.ndarray, g: Grid) -> np.ndarray:
    """Per-QoI relative error: |dn|/n, |du|/max(|u|, sqrt(T_par/m)), |dTperp|/Tperp, |dTpar|/Tpar."""
    q_ref = np.asarray(q_ref, np.float64)
    q = np.asarray(q, np.float64)
    scale = np.stack([np.abs(q_ref[..., 0]),
                      np.maximum(np.abs(q_ref[..., 1]), np.sqrt(np.abs(q_ref[..., 3]) / g.mass)),
                      np.abs(q_ref[..., 2]), np.abs(q_ref[..., 3])], axis=-1)
    return np.abs(q - q_ref) / scale
