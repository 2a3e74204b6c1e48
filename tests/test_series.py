"""Host logic of incremental training (Section IV-D): the column-random-index selection
of training rows and the drifting synthetic series (CPU)."""
import numpy as np
import pytest

from oracle import grid, moments
from paper_2212_10733_amd import synth


def colrandind(*a, **k):
    from paper_2212_10733_amd import train      # imports the binding module (no device use)
    return train.colrandind(*a, **k)


@pytest.fixture(autouse=True)
def _needs_binding():
    pytest.importorskip("paper_2212_10733_amd.train")


def test_colrandind_one_row_per_node():
    planes, nodes = 8, 5000
    idx = colrandind(planes, nodes, seed=3)
    assert idx.shape == (nodes,) and idx.dtype == np.int64
    assert np.array_equal(idx % nodes, np.arange(nodes))          # node m, in node order
    r = idx // nodes
    assert r.min() >= 0 and r.max() < planes
    # the plane of each node is uniform over the planes (chi-square, 7 d.o.f., p ~ 1e-6)
    cnt = np.bincount(r, minlength=planes)
    chi2 = ((cnt - nodes / planes) ** 2 / (nodes / planes)).sum()
    assert chi2 < 40
    assert np.array_equal(colrandind(planes, nodes, seed=3), idx)
    assert not np.array_equal(colrandind(planes, nodes, seed=4), idx)
    assert np.array_equal(colrandind(1, 7), np.arange(7))
    assert colrandind(3, 0).shape == (0,)
    with pytest.raises(ValueError):
        colrandind(0, 5)


def test_series_drifts_and_starts_at_the_plain_generator():
    F0 = synth.series(0, 2, 64)
    assert np.array_equal(F0, synth.histograms(128, seed=synth.SEED_SERIES))
    g = grid.make_grid()
    u = []
    for t in range(3):
        F = synth.histograms(512, seed=synth.SEED_SERIES, shift=synth.series_shift(t)).astype(np.float64)
        u.append(np.median(moments.qoi(F, g)[:, 1]))
    # the bump centres move by +0.15 in v_par per step: the median mean velocity follows
    assert 0.1 < u[1] - u[0] < 0.2 and 0.1 < u[2] - u[1] < 0.2
