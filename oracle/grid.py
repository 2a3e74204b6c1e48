"""Velocity grid, cell volumes and the moment basis (Section II, Eq. 1-4).

A histogram is f[j, i] with j indexing v_perp (rows) and i indexing v_par (columns).
The four moment constraints are written in the u-free basis

    phi_0 = 1, phi_1 = v_par / V_par, phi_2 = (v_perp / V_perp)^2, phi_3 = (v_par / V_par)^2

with V_par = max(|v_par|) and V_perp = max(|v_perp|) over the grid extent.  The discrete
constraint matrix is A[k, (j, i)] = vol[j, i] * phi_k(i, j).  Matching these four raw
moments is equivalent to matching n, u_par, T_perp and T_par, since
(v_par - u)^2 = v_par^2 - 2 u v_par + u^2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Grid:
    n_par: int
    n_perp: int
    vpar: np.ndarray      # (n_par,)
    vperp: np.ndarray     # (n_perp,)
    vol: np.ndarray       # (n_perp, n_par)
    mass: float
    Vpar: float
    Vperp: float

    @property
    def N(self) -> int:
        return self.n_par * self.n_perp

    def basis(self) -> np.ndarray:
        """phi_k on the grid, shape (4, n_perp, n_par)."""
        a = self.vpar / self.Vpar
        c = self.vperp / self.Vperp
        P = np.empty((4, self.n_perp, self.n_par))
        P[0] = 1.0
        P[1] = a[None, :]
        P[2] = (c * c)[:, None]
        P[3] = (a * a)[None, :]
        return P

    def A(self) -> np.ndarray:
        """Constraint matrix, shape (4, N), columns in row-major (j, i) order."""
        return (self.vol[None] * self.basis()).reshape(4, self.N)


def make_grid(n_par: int = 39, n_perp: int = 39, vpar_lo: float = -4.0, vpar_hi: float = 4.0,
              vperp_lo: float = 0.0, vperp_hi: float = 4.0, vol=None, mass: float = 1.0) -> Grid:
    """Uniform grid v_par_i = lo + i * dv_par, dv_par = (hi - lo) / (n_par - 1) (same for v_perp).

    `vol` is None (every cell gets dv_par * dv_perp), the string 'jacobian'
    (dv_par * dv_perp * max(v_perp_j, dv_perp / 4)), or an explicit (n_perp, n_par) array.
    """
    dpar = (vpar_hi - vpar_lo) / (n_par - 1)
    dperp = (vperp_hi - vperp_lo) / (n_perp - 1)
    vpar = vpar_lo + np.arange(n_par) * dpar
    vperp = vperp_lo + np.arange(n_perp) * dperp
    if vol is None:
        V = np.full((n_perp, n_par), dpar * dperp)
    elif isinstance(vol, str) and vol == "jacobian":
        V = np.repeat((dpar * dperp * np.maximum(vperp, dperp / 4))[:, None], n_par, axis=1)
    else:
        V = np.asarray(vol, dtype=np.float64).reshape(n_perp, n_par).copy()
    return Grid(n_par, n_perp, vpar, vperp, V, float(mass),
                max(abs(vpar_lo), abs(vpar_hi)), max(abs(vperp_lo), abs(vperp_hi)))
