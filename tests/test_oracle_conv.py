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


def test_training_gradients_match_torch_autograd():
    """Forward and backward of the FP64 convolutional model against torch autograd (CPU,
    FP64) on the same weights, with an extra dL/dz; and central differences on samples."""
    rng = np.random.default_rng(53)
    W = synth.conv_ae_weights(3)
    for k in ("c1b", "c2b", "fb", "db", "t1b", "t2b"):
        W[k] = rng.normal(0, 0.05, W[k].shape).astype(np.float32)
    B = 5
    X = rng.standard_normal((B, 1521))
    cache = conv.forward_train(X, W)
    dxh = 2 * (cache["xh"] - X) / X.size
    dz = rng.standard_normal((B, 16)) * 1e-3
    g = conv.backward(cache, W, dxh, dz)
    t = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in W.items()}
    xt = t64(X.reshape(B, 1, 39, 39))
    h1 = torch.relu(Fn.conv2d(xt, t["c1w"], t["c1b"], stride=2, padding=1))
    h2 = torch.relu(Fn.conv2d(h1, t["c2w"], t["c2b"], stride=2, padding=1)).reshape(B, -1)
    zt = h2 @ t["fw"].T + t["fb"]
    h4 = torch.relu(zt @ t["dw"].T + t["db"]).reshape(B, 64, 10, 10)
    h5 = torch.relu(Fn.conv_transpose2d(h4, t["t1w"], t["t1b"], stride=2, padding=1, output_padding=1))
    xht = Fn.conv_transpose2d(h5, t["t2w"], t["t2b"], stride=2, padding=1).reshape(B, -1)
    assert np.allclose(cache["xh"], xht.detach().numpy(), rtol=1e-12, atol=1e-12)
    (((xht - t64(X)) ** 2).mean() + (zt * t64(dz)).sum()).backward()
    for k in W:
        ref = t[k].grad.numpy()
        assert np.allclose(g[k], ref, rtol=1e-9, atol=1e-12 * (np.abs(ref).max() + 1e-30)), k
    # central differences of the FP64 loss (without the dz term) at a few coordinates
    g0 = conv.backward(cache, W, dxh)
    W64 = {k: v.astype(np.float64) for k, v in W.items()}
    for k in ("c1w", "c2w", "fw", "t1w", "t2b"):
        idx = tuple(rng.integers(0, s) for s in W64[k].shape)
        Wp = {kk: vv.copy() for kk, vv in W64.items()}
        Wm = {kk: vv.copy() for kk, vv in W64.items()}
        hstep = 1e-6
        Wp[k][idx] += hstep
        Wm[k][idx] -= hstep
        fd = (conv.loss(X, Wp) - conv.loss(X, Wm)) / (2 * hstep)
        assert abs(g0[k][idx] - fd) <= 1e-4 * max(abs(fd), 1e-8) + 1e-11, (k, g0[k][idx], fd)   # ReLU kinks


def test_plain_fp64_model_matches_torch_and_training_forward():
    """encode64 / decode64 (the reference the BF16 form's error is stated against) against
    torch's CPU FP64 layers on the same weights, and against the training forward pass on
    the same z-scored rows; the z-scoring divides by sigma in FP64."""
    F = synth.histograms(5, seed=54, dtype=np.float64)
    W = synth.conv_ae_weights()
    rng = np.random.default_rng(54)
    for k in ("c1b", "c2b", "fb", "db", "t1b", "t2b"):
        W[k] = rng.normal(0, 0.05, W[k].shape).astype(np.float32)
    mu, sd = oracle.ae.norm_stats(F)
    z = conv.encode64(F, mu, sd, W)
    X = (F.reshape(5, -1) - mu) / sd
    Wt = {k: t64(v) for k, v in W.items()}
    h1 = torch.relu(Fn.conv2d(t64(X.reshape(5, 1, 39, 39)), Wt["c1w"], Wt["c1b"], stride=2, padding=1))
    h2 = torch.relu(Fn.conv2d(h1, Wt["c2w"], Wt["c2b"], stride=2, padding=1))
    zt = (h2.reshape(5, -1) @ Wt["fw"].T + Wt["fb"]).numpy()
    assert np.allclose(z, zt, rtol=1e-12, atol=1e-12 * np.abs(zt).max())
    cache = conv.forward_train(X, W)
    assert np.allclose(z, cache["z"], rtol=1e-13, atol=1e-13 * np.abs(zt).max())
    fh = conv.decode64(cache["z"], W, mu, sd)
    assert np.allclose(fh, sd * cache["xh"] + mu, rtol=1e-12, atol=1e-12 * np.abs(fh).max())
    # the decoder's z -> y part against torch directly
    hd = torch.relu(t64(cache["z"]) @ Wt["dw"].T + Wt["db"]).reshape(5, 64, 10, 10)
    h3 = torch.relu(Fn.conv_transpose2d(hd, Wt["t1w"], Wt["t1b"], stride=2, padding=1, output_padding=1))
    y = Fn.conv_transpose2d(h3, Wt["t2w"], Wt["t2b"], stride=2, padding=1).reshape(5, -1).numpy()
    assert np.allclose((fh - mu) / sd, y, rtol=1e-10, atol=1e-11 * np.abs(y).max())


def test_bf16_training_form():
    """The BF16 training form of the convolutional model: its forward pass against torch's
    CPU FP64 layers fed torch's own bfloat16 conversion of both operands of every product
    (biases unrounded); an identity rounding gives the FP64 model bit for bit; its gradients
    are close to the FP64 gradients (bfloat16 operands: about 2^-9 relative per operand, and
    ReLU masks that flip where a pre-activation's sign does) but not equal."""
    rng = np.random.default_rng(55)
    W = synth.conv_ae_weights(5)
    for k in ("c1b", "c2b", "fb", "db", "t1b", "t2b"):
        W[k] = rng.normal(0, 0.05, W[k].shape).astype(np.float32)
    B = 4
    X = rng.standard_normal((B, 1521))
    c16 = conv.forward_train(X, W, rnd=oracle.ae.bf16)

    def tb(a):
        return torch.from_numpy(np.asarray(a, np.float64)).to(torch.bfloat16).to(torch.float64)

    Wt = {k: t64(v) for k, v in W.items()}
    h1 = torch.relu(Fn.conv2d(tb(X.reshape(B, 1, 39, 39)), tb(W["c1w"]), Wt["c1b"], stride=2, padding=1))
    h2 = torch.relu(Fn.conv2d(tb(h1), tb(W["c2w"]), Wt["c2b"], stride=2, padding=1)).reshape(B, -1)
    z = tb(h2) @ tb(W["fw"]).T + Wt["fb"]
    h4 = torch.relu(tb(z) @ tb(W["dw"]).T + Wt["db"]).reshape(B, 64, 10, 10)
    h5 = torch.relu(Fn.conv_transpose2d(tb(h4), tb(W["t1w"]), Wt["t1b"], stride=2, padding=1, output_padding=1))
    xh = Fn.conv_transpose2d(tb(h5), tb(W["t2w"]), Wt["t2b"], stride=2, padding=1).reshape(B, -1).numpy()
    assert np.allclose(c16["z"], z.numpy(), rtol=1e-12, atol=1e-12 * np.abs(z.numpy()).max())
    assert np.allclose(c16["xh"], xh, rtol=1e-10, atol=1e-10 * np.abs(xh).max())
    c64 = conv.forward_train(X, W)
    same = conv.forward_train(X, W, rnd=lambda a: np.asarray(a, np.float64))
    assert np.array_equal(same["xh"], c64["xh"])
    dxh = 2 * (c64["xh"] - X) / X.size
    g64 = conv.backward(c64, W, dxh)
    g16 = conv.backward(c16, W, 2 * (c16["xh"] - X) / X.size, rnd=oracle.ae.bf16)
    for k in g64:
        rel = np.linalg.norm(g16[k] - g64[k]) / np.linalg.norm(g64[k])
        assert 1e-6 < rel < 1e-1, (k, rel)
