"""The convolutional autoencoder of the oracle (BF16 form, 39 x 39 grids) against torch's
CPU FP64 convolution routines and exact rational arithmetic (CPU)."""
from fractions import Fraction

import numpy as np
import torch
import torch.nn.functional as Fn

import oracle
from oracle import conv
from paper_2212_10733_amd import synth


def t64(a):
    return torch.from_numpy(np.asarray(a, np.float64))


def rn32(fr: Fraction) -> np.float32:
    """Nearest FP32 value to a rational (ties to even), from the neighbours of a guess."""
    x0 = np.float32(float(fr))
    cands = [np.nextafter(x0, np.float32(-np.inf)), x0, np.nextafter(x0, np.float32(np.inf))]
    dist = [abs(Fraction(float(v)) - fr) for v in cands]
    best = min(dist)
    ties = [v for v, d in zip(cands, dist) if d == best]
    return ties[0] if len(ties) == 1 else [v for v in ties if (np.float32(v).view(np.uint32) & 1) == 0][0]


def test_shapes_and_parameter_count():
    W = synth.conv_ae_weights()
    assert sum(v.size for v in W.values()) == 248785
    assert all(W[k].shape == s for k, s in synth.CONV_SHAPES.items())


def test_convolutions_match_torch():
    rng = np.random.default_rng(50)
    x = rng.standard_normal((3, 32, 20, 20))
    w = rng.standard_normal((64, 32, 3, 3))
    b = rng.standard_normal(64)
    got = conv.conv2d_s2(x, w, b)
    want = Fn.conv2d(t64(x), t64(w), t64(b), stride=2, padding=1).numpy()
    assert got.shape == (3, 64, 10, 10) and np.allclose(got, want, rtol=1e-13, atol=1e-12)
    xd = rng.standard_normal((3, 64, 10, 10))
    wt = rng.standard_normal((64, 32, 3, 3))
    bt = rng.standard_normal(32)
    got = conv.conv_t2d_s2(xd, wt, bt, 20)
    want = Fn.conv_transpose2d(t64(xd), t64(wt), t64(bt), stride=2, padding=1, output_padding=1).numpy()
    assert got.shape == (3, 32, 20, 20) and np.allclose(got, want, rtol=1e-13, atol=1e-12)
    x3 = rng.standard_normal((2, 32, 20, 20))
    w3 = rng.standard_normal((32, 1, 3, 3))
    got = conv.conv_t2d_s2(x3, w3, np.array([0.25]), 39)
    want = Fn.conv_transpose2d(t64(x3), t64(w3), t64([0.25]), stride=2, padding=1).numpy()
    assert got.shape == (2, 1, 39, 39) and np.allclose(got, want, rtol=1e-13, atol=1e-12)


def test_first_layer_is_the_fp32_chain():
    """Against torch FP64 (about nine FP32 roundings apart) and, for sampled outputs,
    against the chain evaluated in exact rational arithmetic."""
    rng = np.random.default_rng(51)
    x32 = rng.standard_normal((2, 39, 39)).astype(np.float32)
    w = rng.standard_normal((32, 1, 3, 3)).astype(np.float32)
    b = (0.1 * rng.standard_normal(32)).astype(np.float32)
    got = conv.conv1_fp32(x32, w, b)
    ref = np.maximum(Fn.conv2d(t64(x32[:, None]), t64(w), t64(b), stride=2, padding=1).numpy(), 0)
    scale = Fn.conv2d(t64(np.abs(x32[:, None])), t64(np.abs(w)), t64(np.abs(b)), stride=2, padding=1).numpy()
    assert np.all(np.abs(got - ref) <= 10 * 2.0 ** -24 * scale)
    for (h, c, oy, ox) in [(0, 0, 0, 0), (1, 31, 19, 19), (0, 7, 0, 13), (1, 3, 11, 0), (0, 12, 9, 10)]:
        s = np.float32(b[c])
        for ky in range(3):
            for kx in range(3):
                iy, ix = 2 * oy - 1 + ky, 2 * ox - 1 + kx
                if 0 <= iy < 39 and 0 <= ix < 39:
                    s = rn32(Fraction(float(x32[h, iy, ix])) * Fraction(float(w[c, 0, ky, kx])) + Fraction(float(s)))
        assert got[h, c, oy, ox] == max(s, np.float32(0)), (h, c, oy, ox)


def test_bf16_form_is_close_to_the_fp64_model():
    """Encoder and decoder of the BF16 form against the same model in FP64 throughout:
    close (the bfloat16 roundings of two layers' operands) but not equal."""
    F = synth.histograms(6, seed=52, dtype=np.float32)
    W = synth.conv_ae_weights()
    mu, sd = oracle.ae.norm_stats(F.astype(np.float64))
    mu32, sd32 = mu.astype(np.float32), sd.astype(np.float32)
    rsd32 = np.float32(1) / sd32
    z = conv.encode_bf16(F, mu32, rsd32, W)
    X = torch.from_numpy(((F.astype(np.float64).reshape(6, -1) - mu32) * rsd32).reshape(6, 1, 39, 39))
    Wt = {k: t64(v) for k, v in W.items()}
    h1 = torch.relu(Fn.conv2d(X, Wt["c1w"], Wt["c1b"], stride=2, padding=1))
    h2 = torch.relu(Fn.conv2d(h1, Wt["c2w"], Wt["c2b"], stride=2, padding=1))
    z64 = (h2.reshape(6, -1) @ Wt["fw"].T + Wt["fb"]).numpy()
    rel = np.abs(z - z64).max() / np.abs(z64).max()
    assert 1e-6 < rel < 3e-2, rel
    Zh = z.astype(np.float32)
    fh = conv.decode_bf16(Zh, W, mu32, sd32)
    hd = torch.relu(t64(Zh) @ Wt["dw"].T + Wt["db"]).reshape(6, 64, 10, 10)
    h3 = torch.relu(Fn.conv_transpose2d(hd, Wt["t1w"], Wt["t1b"], stride=2, padding=1, output_padding=1))
    y = Fn.conv_transpose2d(h3, Wt["t2w"], Wt["t2b"], stride=2, padding=1).reshape(6, -1).numpy()
    f64 = sd32.astype(np.float64) * y + mu32
    rel = np.abs(fh - f64).max() / np.abs(f64 - mu32).max()
    assert 1e-6 < rel < 3e-2, rel
