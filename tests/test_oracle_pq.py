"""Pins of the oracle's product quantizer (Section III Stage 3, Section IV-E)."""
import json
import os

import numpy as np
import pytest

from oracle import pq
from paper_2212_10733_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_sizes.json")


def brute_nearest_value(z, C):
    # the nearest centroid value, exact midpoints to the lower value, by exhaustive comparison
    # in exact arithmetic
    from fractions import Fraction
    out = []
    for v in z:
        fv = Fraction(float(v))
        vals = sorted(set(Fraction(float(c)) for c in C))
        out.append(float(min(vals, key=lambda c: (abs(fv - c), c))))
    return np.array(out)


def test_encode_is_nearest_centroid_lower_tie():
    C = np.sort(np.random.default_rng(0).normal(size=32)).astype(np.float32)
    C[5] = C[6]                               # duplicate centroid
    beta = (C[:-1].astype(np.float64) + C[1:].astype(np.float64)) * 0.5
    z = np.concatenate([np.random.default_rng(1).normal(size=300),
                        beta[::3], [C[0] - 1, C[-1] + 1], C[::4]]).astype(np.float32)
    got = pq.encode(z[:, None], C[None, :])[:, 0]
    assert np.array_equal(C[got].astype(np.float64), brute_nearest_value(z, C))
    # exact midpoints between distinct neighbours go to the lower centroid
    mids = beta[(C[1:] != C[:-1])]
    exact = mids[mids.astype(np.float32).astype(np.float64) == mids].astype(np.float32)
    assert exact.size > 0
    code = pq.encode(exact[:, None], C[None, :])[:, 0]
    assert np.all(C[code].astype(np.float64) < exact.astype(np.float64))


def kmeans_dp(x, k):
    """Exact 1-D k-means optimum by dynamic programming over sorted prefixes."""
    x = np.sort(np.asarray(x, np.float64))
    n = x.size
    def sse(a, b):
        seg = x[a:b + 1]
        return float(((seg - seg.mean()) ** 2).sum())
    INF = float("inf")
    D = [[INF] * (n + 1) for _ in range(k + 1)]
    D[0][0] = 0.0
    for m in range(1, k + 1):
        for i in range(m, n + 1):
            D[m][i] = min(D[m - 1][j] + sse(j, i - 1) for j in range(m - 1, i))
    return D[k][n]


def test_lloyd_fixed_point_invariants():
    s = synth.latents(2000, 1, seed=3)[:, 0]
    C, updates = pq.fit_1d(s, 16)
    assert updates <= 25
    assert np.all(np.diff(C) >= 0)
    a = pq.assign_1d(s, C)
    ok = 0
    for c in range(16):
        m = s[a == c].astype(np.float64)
        if m.size:
            ok += np.isclose(C[c], m.mean(), rtol=1e-14)
    assert ok == np.unique(a).size
    # every member's nearest centroid is its own
    d = np.abs(s.astype(np.float64)[:, None] - C[None, :])
    assert np.all(d[np.arange(s.size), a] <= d.min(axis=1) + 1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_lloyd_vs_dynamic_programming_optimum(seed):
    rng = np.random.default_rng(seed)
    if seed < 3:   # well separated clusters: Lloyd from quantile init reaches the optimum
        x = np.concatenate([rng.normal(c, 0.05, 3) for c in (0.0, 5.0, 10.0, 20.0)])
    else:
        x = rng.normal(size=12)
    C, _ = pq.fit_1d(x, 4)
    opt = kmeans_dp(x, 4)
    cost = pq.kmeans_cost(x, C)
    assert cost >= opt - 1e-12
    if seed < 3:
        assert cost == pytest.approx(opt, rel=1e-12)


def test_quantile_init_and_empty_cluster_keeps_centroid():
    s = np.array([0.0, 0.0, 0.0, 0.0, 1.0])
    C, _ = pq.fit_1d(s, 4)     # init at sorted[(2c+1)*5//8] = [0, 0, 0, 1]
    assert C[-1] == 1.0 and C[0] == 0.0
    assert np.all(np.diff(C) >= 0)


def test_fit_uses_every_kth_row():
    Z = synth.latents(64, 2, seed=4)
    C1 = pq.fit(Z, bits=3, sample_every=4)
    C2 = pq.fit(Z[::4], bits=3, sample_every=1)
    assert np.array_equal(C1, C2)
    assert C1.dtype == np.float32 and C1.shape == (2, 8)


def test_paper_size_accounting():
    gold = json.load(open(GOLD))
    lb = gold["latent_bits_per_image"]
    codes = np.zeros((1, lb["L"]), np.uint8)
    assert codes.shape[1] * lb["B"] == lb["bits"]
    t = gold["pq_table_bytes"]
    C = pq.fit(synth.latents(256, t["L"], seed=5), bits=int(np.log2(t["k"])))
    assert C.nbytes == t["bytes"] == 16 * t["k"]
    w = gold["tied_ae_weight_bytes"]
    Wt = np.zeros((w["latent"], w["n_perp"] * w["n_par"]), np.float32)
    assert Wt.nbytes == w["bytes"]


def test_assignment_is_the_midpoint_count():
    # the binary search equals the literal count #{c : beta_c < z}, NaN counting none
    rng = np.random.default_rng(9)
    C = np.sort(rng.normal(size=64))
    C[10] = C[11]
    beta = pq.midpoints(C)
    z = np.concatenate([rng.normal(size=2000), beta, [np.inf, -np.inf, np.nan]])
    assert np.array_equal(pq.assign_1d(z, C), (beta[None, :] < z[:, None]).sum(axis=1))
