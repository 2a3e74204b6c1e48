"""The output container (Section III, end of Stage 5: header, weights, codes, PQ table,
residual bytes, multipliers) and its order-0 rANS coder: host logic, no GPU."""
import math
import struct

import numpy as np
import pytest

from paper_2212_10733_amd import synth


@pytest.fixture(scope="module")
def H():
    from paper_2212_10733_amd import hcz
    return hcz


def entropy_bytes(a: np.ndarray) -> float:
    c = np.bincount(a, minlength=256).astype(np.float64)
    p = c[c > 0] / a.size
    return float(-(p * np.log2(p)).sum() * a.size / 8)


def test_rans_round_trips_and_is_near_the_entropy(H):
    rng = np.random.default_rng(80)
    cases = [np.zeros(0, np.uint8), np.full(5000, 9, np.uint8), rng.integers(0, 256, 200000, dtype=np.uint8),
             rng.geometric(0.2, 300000).clip(0, 255).astype(np.uint8),
             np.frombuffer(rng.standard_normal(50000).astype(np.float32).tobytes(), np.uint8)]
    for a in cases:
        e = H.rans_encode(a)
        assert np.array_equal(H.rans_decode(e, a.size), a)
        if a.size:
            # 12-bit frequencies cost at most a fraction of a percent over order-0 entropy
            assert len(e) <= 1.01 * entropy_bytes(a) + 600 + 0.002 * a.size


def test_rans_rejects_malformed_blocks(H):
    a = np.random.default_rng(81).geometric(0.3, 10000).clip(0, 255).astype(np.uint8)
    e = H.rans_encode(a)
    with pytest.raises(RuntimeError):
        H.rans_decode(e[:-3], a.size)                    # truncated
    with pytest.raises(RuntimeError):
        H.rans_decode(e, a.size + 1)                     # wrong length
    bad = bytearray(e)
    bad[8 + 2 * int(a[0])] ^= 0x01                       # frequency table no longer sums to 4096
    with pytest.raises(RuntimeError):
        H.rans_decode(bytes(bad), a.size)
    bad = bytearray(e)
    bad[-1] ^= 0x5a                                      # payload corruption: final state check
    try:
        out = H.rans_decode(bytes(bad), a.size)
        assert not np.array_equal(out, a)
    except RuntimeError:
        pass


def fake_batch(Hn, N, rng, lam_dtype=np.float64):
    sizes = rng.integers(0, 300, Hn).astype(np.uint64)
    sizes[rng.random(Hn) < 0.2] = 0
    off = np.zeros(Hn + 1, np.uint64)
    off[1:] = np.cumsum(sizes)
    return dict(flags=rng.integers(0, 32, Hn).astype(np.uint8), res_offset=off,
                res_bytes=rng.geometric(0.1, int(off[-1])).clip(0, 255).astype(np.uint8),
                lam=rng.standard_normal((Hn, 4)).astype(lam_dtype))


@pytest.mark.parametrize("entropy", [False, True])
@pytest.mark.parametrize("with_model", [False, True])
def test_container_round_trip(H, entropy, with_model):
    rng = np.random.default_rng(82)
    Hn, N = 300, 1521
    b = fake_batch(Hn, N, rng, np.float32 if with_model else np.float64)
    kw = {}
    if with_model:
        W = synth.dense_ae_weights()
        kw = dict(codes=rng.geometric(0.05, (Hn, 16)).clip(0, 255).astype(np.uint8),
                  centroids=np.sort(rng.standard_normal((16, 256)).astype(np.float32), axis=1),
                  weights=np.concatenate([W[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")]),
                  norm_mean=rng.random(N).astype(np.float32), norm_std=rng.random(N).astype(np.float32) + 0.1,
                  arch="dense", compute="bf16")
    buf = H.container_pack(39, 39, entropy=entropy, **b, **kw)
    assert buf[:4] == b"HCZ1"
    hdr = struct.unpack("<4sHBBQHHIQQI", buf[:44])
    assert hdr[4] == Hn and hdr[5] == 39 and hdr[9] == len(buf)
    d = H.container_unpack(buf)
    assert d["H"] == Hn and d["entropy"] == entropy
    for k in ("flags", "res_offset", "res_bytes", "lam"):
        assert d[k].dtype == np.asarray(b[k]).dtype and np.array_equal(d[k], b[k]), k
    if with_model:
        assert d["arch"] == "dense" and d["compute"] == "bf16"
        for k in ("codes", "centroids", "weights", "norm_mean", "norm_std"):
            assert np.array_equal(d[k], kw[k]), k
    else:
        assert d["arch"] is None
    if entropy:
        plain = H.container_pack(39, 39, entropy=False, **b, **kw)
        assert len(buf) < len(plain)


def test_container_rejects_damage(H):
    rng = np.random.default_rng(83)
    b = fake_batch(50, 1521, rng)
    buf = H.container_pack(39, 39, entropy=True, **b)
    with pytest.raises(RuntimeError):
        H.container_unpack(buf[:30])                     # shorter than the header
    with pytest.raises(RuntimeError):
        H.container_unpack(buf[:len(buf) - 8])           # total size beyond the buffer
    bad = bytearray(buf)
    bad[9] ^= 1                                          # H changed: header checksum
    with pytest.raises(RuntimeError):
        H.container_unpack(bytes(bad))
    bad = bytearray(buf)
    bad[48 + 50 + 1] ^= 0xff                             # a record size (after 50 flags): sizes inconsistent
    with pytest.raises(RuntimeError):
        H.container_unpack(bytes(bad))
