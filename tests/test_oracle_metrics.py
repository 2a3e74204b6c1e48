"""Pins of the oracle's error and size metrics (Eq. 7 and Section IV-A) and of its z-score
statistics (Section IV-D), against hand-computed values, closed forms and the paper's
printed sizes."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ae, grid, metrics, pipeline

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_sizes.json")


def test_nrmse_hand_computed():
    # u = 0, 1, 2, 3 and f off by 2 in one place: sqrt(4 / 4) / (3 - 0) = 1/3
    assert metrics.nrmse([0, 1, 2, 3], [0, 1, 2, 5]) == pytest.approx(1 / 3, rel=1e-15)
    # u's range, not f's, normalises: the same error against a range of 10
    assert metrics.nrmse([0, 10, 5, 5], [0, 10, 5, 7]) == pytest.approx(math.sqrt(1.0) / 10, rel=1e-15)
    # an error spread over every element: sqrt(sum 0.5^2 / 8) / 7 = 0.5 / 7
    u = np.arange(8.0)
    assert metrics.nrmse(u, u + 0.5) == pytest.approx(0.5 / 7, rel=1e-15)
    assert metrics.nrmse(u, u) == 0.0


def test_nrmse_invariances_and_bound_relation():
    """NRMSE is unchanged by a common shift and a positive scale of u and f, symmetric in
    the sign of the error, and NRMSE(u, f) <= tau is the same statement as the per-image
    bound ||u - f||_2 <= tau sqrt(N) (max u - min u) of the NRMSE bound mode."""
    rng = np.random.default_rng(3)
    u = rng.random((7, 5))
    f = u + 1e-3 * rng.standard_normal(u.shape)
    e = metrics.nrmse(u, f)
    assert metrics.nrmse(3.5 * u - 2.0, 3.5 * f - 2.0) == pytest.approx(e, rel=1e-12)
    assert metrics.nrmse(u, 2 * u - f) == pytest.approx(e, rel=1e-12)
    g = grid.make_grid(5, 7)
    F = u[None]
    th = pipeline.tau_h(F, pipeline.Params(tau=e, tau_mode="nrmse"))[0]
    assert np.linalg.norm(u - f) == pytest.approx(th, rel=1e-12)
    assert g.N == u.size


def test_compressed_bytes_paper_sizes_and_hand_count():
    gold = json.load(open(GOLD))
    lb = gold["latent_bits_per_image"]
    # an L = 4, B = 4 latent takes L x B = 16 bits, 2 bytes per image (Section III Stage 3):
    # with nothing else stored, 1,000 images cost 2,000 bytes of codes plus one flag byte each
    assert metrics.compressed_bytes(1000, lb["L"], lb["B"], 0, lam_bytes=0, header=0) == 1000 * lb["bits"] // 8 + 1000
    pq = gold["pq_table_bytes"]
    tw = gold["tied_ae_weight_bytes"]
    # hand count: 3 images, latent 4 at 4 bits (6 bytes of codes), FP64 multipliers (96),
    # flags (3), 100 residual bytes, the paper's PQ table (256) and tied weights (19,536),
    # and the 44-byte header
    got = metrics.compressed_bytes(3, 4, 4, 100, lam_bytes=8, model_bytes=tw["bytes"], codebook_bytes=pq["bytes"])
    assert got == 6 + 96 + 3 + 100 + 19536 + 256 + 44
    # FP32 multipliers (the paper's production choice) halve that section
    assert got - metrics.compressed_bytes(3, 4, 4, 100, lam_bytes=4, model_bytes=tw["bytes"],
                                          codebook_bytes=pq["bytes"]) == 48
    # codes are packed across images: 5 images of 3 x 3 bits = 45 bits -> 6 bytes
    assert metrics.compressed_bytes(5, 3, 3, 0, lam_bytes=0, header=0) == 6 + 5
    assert metrics.compression_ratio(6000, 1500) == 4.0


def test_norm_stats_closed_form():
    """Per-pixel mean and population std against columns whose statistics are known in
    closed form: 1..n has mean (n+1)/2 and population variance (n^2 - 1)/12 (the sample
    variance would be n(n+1)/12); +-c alternating has mean 0 and std c; a constant pixel
    gets the floor 1e-12 times the largest std."""
    n = 10
    F = np.zeros((n, 2, 2))
    F[:, 0, 0] = np.arange(1, n + 1)
    F[:, 0, 1] = np.where(np.arange(n) % 2 == 0, 3.0, -3.0)
    F[:, 1, 0] = 7.25
    F[:, 1, 1] = 2.0 * np.arange(1, n + 1) + 5.0           # affine image of 1..n
    mu, sd = ae.norm_stats(F)
    assert mu[0] == pytest.approx((n + 1) / 2, rel=1e-15)
    assert sd[0] == pytest.approx(math.sqrt((n * n - 1) / 12), rel=1e-14)
    assert mu[1] == 0.0 and sd[1] == pytest.approx(3.0, rel=1e-15)
    assert mu[2] == 7.25
    assert sd[2] == pytest.approx(1e-12 * 2.0 * math.sqrt((n * n - 1) / 12), rel=1e-12)
    assert mu[3] == pytest.approx(2.0 * (n + 1) / 2 + 5.0, rel=1e-15)
    assert sd[3] == pytest.approx(2.0 * math.sqrt((n * n - 1) / 12), rel=1e-14)
