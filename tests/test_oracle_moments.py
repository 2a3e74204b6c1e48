"""Pins of the oracle's moments and QoIs (Eq. 1-4) against closed forms."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import grid, moments


def test_delta_histogram_closed_form():
    # A single non-zero cell: n = w vol, u_par = v_par_i, T_perp = m v_perp_j^2 / 2, T_par = 0.
    g = grid.make_grid(39, 39, mass=2.5)
    for (j, i) in [(0, 0), (7, 30), (38, 19), (20, 5)]:
        f = np.zeros((39, 39))
        f[j, i] = 3.0
        n, u, tperp, tpar = moments.qoi(f, g)
        assert n == pytest.approx(3.0 * g.vol[j, i], rel=1e-15)
        assert u == pytest.approx(g.vpar[i], rel=1e-14, abs=1e-15)
        assert tperp == pytest.approx(0.5 * 2.5 * g.vperp[j] ** 2, rel=1e-14, abs=1e-15)
        assert abs(tpar) <= 1e-13 * max(1.0, 2.5 * g.vpar[i] ** 2)


def test_uniform_histogram_exact_rationals():
    # f = 1 on the 39x39 grid v_par = -4 + 8i/38, v_perp = 4j/38 (m = 1):
    # u_par = 0, T_perp = (1/2) mean_j v_perp_j^2, T_par = (1/2) mean_i v_par_i^2 (Faulhaber sums).
    g = grid.make_grid(39, 39)
    f = np.ones((39, 39))
    n, u, tperp, tpar = moments.qoi(f, g)
    tperp_exact = Fraction(1, 2) * sum(Fraction(4 * j, 38) ** 2 for j in range(39)) / 39
    tpar_exact = Fraction(1, 2) * sum((Fraction(-4) + Fraction(8 * i, 38)) ** 2 for i in range(39)) / 39
    assert n == pytest.approx(1521 * (8 / 38) * (4 / 38), rel=1e-14)
    assert abs(u) < 1e-14
    assert tperp == pytest.approx(float(tperp_exact), rel=1e-14)
    assert tpar == pytest.approx(float(tpar_exact), rel=1e-14)


def test_mirror_symmetry_gives_zero_flow():
    g = grid.make_grid(39, 39)
    rng = np.random.default_rng(0)
    half = rng.random((39, 20))
    f = np.concatenate([half, half[:, :19][:, ::-1]], axis=1)
    assert np.allclose(f, f[:, ::-1])
    _, u, _, _ = moments.qoi(f, g)
    assert abs(u) < 1e-14


def test_linearity():
    g = grid.make_grid(39, 39, vol="jacobian")
    rng = np.random.default_rng(1)
    f1, f2 = rng.random((39, 39)), rng.random((39, 39))
    b = moments.moments(2.0 * f1 - 0.5 * f2, g)
    assert np.allclose(b, 2.0 * moments.moments(f1, g) - 0.5 * moments.moments(f2, g), rtol=1e-14, atol=1e-15)


def test_direct_and_moment_forms_agree():
    g = grid.make_grid(33, 37, vpar_lo=-3.0, vpar_hi=3.5, vperp_hi=3.0, vol="jacobian", mass=0.7)
    rng = np.random.default_rng(2)
    f = rng.random((37, 33))
    assert np.allclose(moments.qoi(f, g), moments.qoi_direct(f, g), rtol=1e-12)


def test_basis_scales_are_grid_half_extent():
    g = grid.make_grid(39, 39)
    assert g.Vpar == 4.0 and g.Vperp == 4.0
    P = g.basis()
    assert P[1].max() == pytest.approx(1.0) and P[2].max() == pytest.approx(1.0)
