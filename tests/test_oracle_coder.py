"""Pins of the oracle's multilevel residual coder (Section III Stage 4)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import coder


def test_ladder_literals_are_correctly_rounded_fourth_roots():
    for m, c in enumerate(coder.LADDER_C):
        exact_pow = Fraction(2) ** m                 # c must be the binary64 nearest 2^(m/4)
        lo, hi = np.nextafter(c, 0.0), np.nextafter(c, 4.0)
        mid_lo, mid_hi = (Fraction(lo) + Fraction(c)) / 2, (Fraction(c) + Fraction(hi)) / 2
        assert mid_lo ** 4 < exact_pow < mid_hi ** 4 or (m == 0 and c == 1.0)


def test_layout_39_groups_and_header():
    lay = coder.layout(39, 39)
    assert lay.L == 6 and lay.nlev == 7 and lay.header_bytes == 24
    sizes = [len(J) for J, _ in lay.groups()]
    assert sizes == [4, 5, 7, 20, 85, 279, 1121] and sum(sizes) == 1521
    seen = set()
    for J, I in lay.groups():
        for j, i in zip(J, I):
            seen.add((j, i))
    assert len(seen) == 1521


@pytest.mark.parametrize("n_par,n_perp", [(3, 3), (9, 17), (33, 33), (39, 39), (5, 12), (65, 65)])
def test_layout_is_a_partition(n_par, n_perp):
    lay = coder.layout(n_par, n_perp)
    seen = [(j, i) for J, I in lay.groups() for j, i in zip(J, I)]
    assert len(seen) == len(set(seen)) == n_par * n_perp


def test_dyadic_grid_roundtrip_exact_on_integers():
    lay = coder.layout(17, 9)            # all interpolation weights are 0 or 1/2
    r = np.random.default_rng(0).integers(-1000, 1000, size=(4, 9, 17)).astype(np.float64)
    d = coder.decompose(r, lay)
    assert np.array_equal(coder.recompose(d, lay), r)


def test_roundtrip_39_close():
    lay = coder.layout(39, 39)
    r = np.random.default_rng(1).normal(size=(3, 39, 39))
    d = coder.decompose(r, lay)
    assert np.max(np.abs(coder.recompose(d, lay) - r)) <= 8 * np.finfo(float).eps * np.abs(r).max()


def test_bilinear_function_has_no_details():
    # Interpolation reproduces bilinear functions, so only the coarse nodes carry values.
    lay = coder.layout(17, 9)
    jj, ii = np.meshgrid(np.arange(9.0), np.arange(17.0), indexing="ij")
    r = (3.0 + 2.0 * ii - 5.0 * jj + 0.5 * ii * jj)[None]
    d = coder.decompose(r, lay)
    mask = np.ones((9, 17), bool)
    mask[lay.coarse_J, lay.coarse_I] = False
    assert np.all(d[0][mask] == 0.0)
    lay39 = coder.layout(39, 39)
    jj, ii = np.meshgrid(np.arange(39.0), np.arange(39.0), indexing="ij")
    d = coder.decompose((1.0 + ii + 2 * jj - 0.25 * ii * jj)[None], lay39)
    mask = np.ones((39, 39), bool)
    mask[lay39.coarse_J, lay39.coarse_I] = False
    assert np.max(np.abs(d[0][mask])) < 1e-12


@pytest.mark.parametrize("shape", [(39, 39), (33, 33), (7, 5)])
def test_pointwise_error_bound_and_level0_feasible(shape):
    n_perp, n_par = shape
    lay = coder.layout(n_par, n_perp)
    rng = np.random.default_rng(2)
    r = rng.normal(size=(8, n_perp, n_par)) * rng.uniform(0.1, 10, size=(8, 1, 1))
    d = coder.decompose(r, lay)
    th = rng.uniform(1e-4, 1e-1, size=8) * np.sqrt((r * r).sum((1, 2)))
    d0 = coder.delta0(th, lay)
    for k in (0, 5, 17):
        Dk = coder.ladder(d0, np.full(8, k))
        q = coder.quantize(d, Dk)
        err = np.abs(r - coder.reconstruct(q, Dk, lay)).reshape(8, -1).max(axis=1)
        assert np.all(err <= (lay.L + 1) * Dk / 2 * (1 + 1e-12))
    ok, _, _ = coder.feasible(r, d, d0, coder.SEL_MARGIN * th, lay)
    assert ok.all()


def test_bisection_exit_property_and_brute_force():
    lay = coder.layout(39, 39)
    rng = np.random.default_rng(3)
    r = rng.normal(size=(6, 39, 39))
    th = np.array([1e-3, 1e-2, 1e-1, 0.3, 3.0, 30.0]) * np.sqrt((r * r).sum((1, 2)))
    thr = coder.SEL_MARGIN * th
    d = coder.decompose(r, lay)
    d0 = coder.delta0(th, lay)
    ks, q, rh = coder.bisect(r, d, d0, thr, lay)
    for h in range(6):
        ok, _, _ = coder.feasible(r[h:h + 1], d[h:h + 1], coder.ladder(d0[h:h + 1], ks[h:h + 1]), thr[h:h + 1], lay)
        assert ok[0]
        if ks[h] + 1 < coder.NLADDER:
            ok2, _, _ = coder.feasible(r[h:h + 1], d[h:h + 1], coder.ladder(d0[h:h + 1], ks[h:h + 1] + 1), thr[h:h + 1], lay)
            assert not ok2[0]
        # replay the search path explicitly
        lo, hi = 0, 41
        while hi - lo > 1:
            mid = (lo + hi) // 2
            okm, _, _ = coder.feasible(r[h:h + 1], d[h:h + 1], coder.ladder(d0[h:h + 1], np.array([mid])), thr[h:h + 1], lay)
            lo, hi = (mid, hi) if okm[0] else (lo, mid)
        assert lo == ks[h]
    assert ks[-1] == 40   # a huge bound saturates the ladder


def test_zigzag():
    for q in [0, 1, -1, 2, -2, 12345, -12345, 2 ** 30 - 1, -(2 ** 30)]:
        u = coder.zigzag(q)
        assert u >= 0 and coder.unzigzag(u) == q
        assert u == (((q << 1) ^ (q >> 31)) & 0xFFFFFFFF)


@pytest.mark.parametrize("shape", [(39, 39), (3, 3), (33, 37)])
def test_pack_unpack_identity_and_size(shape):
    n_perp, n_par = shape
    lay = coder.layout(n_par, n_perp)
    rng = np.random.default_rng(4)
    q = rng.integers(-5000, 5000, size=(n_perp, n_par))
    q[lay.coarse_J, lay.coarse_I] = 0    # a zero-width group
    rec = coder.pack(q, 0.123, 7, lay)
    q2, Delta, k = coder.unpack(rec, lay)
    assert np.array_equal(q, q2) and Delta == 0.123 and k == 7
    widths = list(rec[10:10 + lay.nlev])
    assert widths[0] == 0
    assert len(rec) == coder.record_size(widths, lay)
    assert len(rec) % 4 == 0 and lay.header_bytes % 8 == 0


def test_guided_search_against_brute_force():
    """The exponential search from a predicted index followed by bisection, on its own with
    made-up feasibility: for every monotone boundary b (0..40 feasible up to b) and every
    start, it returns b; for arbitrary non-monotone patterns (index 0 always feasible) it
    returns a feasible k whose successor is infeasible or 41, and without a start it is the
    plain bisection."""
    K = coder.NLADDER
    for start in range(K):
        b = np.arange(K)
        got = coder.search(None, np.zeros((K, 1, 1)), None, None, None, start,
                           feasible_at=lambda rows, k: k <= b[rows])
        assert np.array_equal(got, b), start
    rng = np.random.default_rng(9)
    pat = rng.random((500, K)) < rng.random((500, 1))
    pat[:, 0] = True
    for start in (None, 0, 5, 11, 40):
        got = coder.search(None, np.zeros((500, 1, 1)), None, None, None, start,
                           feasible_at=lambda rows, k: pat[rows, k])
        assert np.all(pat[np.arange(500), got])
        nxt = np.minimum(got + 1, K - 1)
        assert np.all((got == K - 1) | ~pat[np.arange(500), nxt])
        if start is None:
            for h in range(500):
                lo, hi = 0, K
                while hi - lo > 1:
                    mid = (lo + hi) // 2
                    lo, hi = (mid, hi) if pat[h, mid] else (lo, mid)
                assert got[h] == lo


def test_guided_search_start_and_agreement_on_residuals():
    """The start index round(4 log2(L+1)) for the grids in use, and on real residuals the
    guided search lands where the bisection does (feasibility is monotone there)."""
    assert coder.search_start(coder.layout(39, 39)) == 11       # L = 6
    assert coder.search_start(coder.layout(3, 3)) == 4          # L = 1
    assert coder.search_start(coder.layout(65, 65)) == 11       # L = 6
    assert coder.search_start(coder.layout(12, 12)) == 9        # L = 4
    lay = coder.layout(39, 39)
    from paper_2212_10733_amd import synth
    F = synth.histograms(40, seed=8, dtype=np.float64)
    rng = np.random.default_rng(4)
    r = F - F.mean(axis=0) + rng.normal(size=F.shape) * 1e-3 * F.max()
    th = np.geomspace(1e-4, 0.5, 40) * np.sqrt((r * r).sum((1, 2)))
    thr = coder.SEL_MARGIN * th
    d = coder.decompose(r, lay)
    d0 = coder.delta0(th, lay)
    kb, qb, rb = coder.bisect(r, d, d0, thr, lay)
    probes = np.zeros(40, np.int64)

    def counted(rows, k):
        probes[rows] += 1
        ok, _, _ = coder.feasible(r[rows], d[rows], coder.ladder(d0[rows], k), thr[rows], lay)
        return ok

    kg = coder.search(None, d, d0, thr, lay, coder.search_start(lay), feasible_at=counted)
    _, qg, rg = coder.search(r, d, d0, thr, lay, coder.search_start(lay))
    assert len(np.unique(kb)) > 5
    # the exit property on real residuals; k* equals the bisection's on most histograms
    # (where feasibility is not monotone each may stop at a different boundary)
    for k in (kg, kb):
        ok, _, _ = coder.feasible(r, d, coder.ladder(d0, k), thr, lay)
        assert ok.all()
        ok1, _, _ = coder.feasible(r, d, coder.ladder(d0, np.minimum(k + 1, 40)), thr, lay)
        assert np.all((k == 40) | ~ok1)
    assert (kg == kb).mean() >= 0.6
    assert np.array_equal(qg, coder.quantize(d, coder.ladder(d0, kg)))
    assert probes.mean() < 4.5
