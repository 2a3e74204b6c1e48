"""Pins of the oracle's autoencoder (Section III Stages 2-3, Eq. 5): library routines,
finite differences and the PCA optimum of a tied linear AE."""
import numpy as np
import pytest
import torch

from oracle import ae
from paper_2212_10733_amd import synth


def small_weights(N=50, hidden=12, latent=4, seed=3):
    W = synth.dense_ae_weights(N, hidden, latent, seed=seed)
    rng = np.random.default_rng(seed)
    for k in ("b1", "b2", "b3", "b4"):   # non-zero biases so they are exercised
        W[k] = rng.normal(0, 0.1, W[k].shape).astype(np.float32)
    return W


def test_forward_matches_torch_linear():
    W = small_weights()
    X = np.random.default_rng(0).normal(size=(7, 50))
    t = {k: torch.tensor(v, dtype=torch.float64) for k, v in W.items()}
    x = torch.tensor(X)
    h = torch.relu(torch.nn.functional.linear(x, t["W1"], t["b1"]))
    z = torch.nn.functional.linear(h, t["W2"], t["b2"])
    h3 = torch.relu(torch.nn.functional.linear(z, t["W3"], t["b3"]))
    xh = torch.nn.functional.linear(h3, t["W4"], t["b4"])
    assert np.allclose(ae.dense_encode(X, W), z.numpy(), rtol=1e-13, atol=1e-13)
    assert np.allclose(ae.dense_decode(z.numpy(), W), xh.numpy(), rtol=1e-13, atol=1e-13)


def test_backward_matches_autograd_and_finite_differences():
    W = {k: v.astype(np.float64) for k, v in small_weights().items()}
    X = np.random.default_rng(1).normal(size=(5, 50))
    g = ae.dense_backward(ae.dense_forward_train(X, W), W)
    t = {k: torch.tensor(v, requires_grad=True) for k, v in W.items()}
    x = torch.tensor(X)
    h = torch.relu(x @ t["W1"].T + t["b1"])
    z = h @ t["W2"].T + t["b2"]
    h3 = torch.relu(z @ t["W3"].T + t["b3"])
    xh = h3 @ t["W4"].T + t["b4"]
    torch.nn.functional.mse_loss(xh, x).backward()
    for k in W:
        assert np.allclose(g[k], t[k].grad.numpy(), rtol=1e-10, atol=1e-13), k
    rng = np.random.default_rng(2)
    eps = 1e-6
    for k in W:
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in W[k].shape)
            Wp = {kk: vv.copy() for kk, vv in W.items()}
            Wm = {kk: vv.copy() for kk, vv in W.items()}
            Wp[k][idx] += eps
            Wm[k][idx] -= eps
            fd = (ae.dense_loss(X, Wp) - ae.dense_loss(X, Wm)) / (2 * eps)
            assert fd == pytest.approx(g[k][idx], rel=1e-5, abs=1e-9), (k, idx)


def test_tied_linear_ae_recovers_pca_subspace():
    # Baldi & Hornik: the MSE optimum of a linear AE spans the top principal subspace.
    rng = np.random.default_rng(4)
    N, L, B = 20, 4, 400
    basis, _ = np.linalg.qr(rng.normal(size=(N, L)))
    X = (rng.normal(size=(B, L)) * np.array([3.0, 2.0, 1.5, 1.0])) @ basis.T
    Wt = rng.normal(0, 0.1, size=(L, N))
    params, state = {"W": Wt}, {}
    for _ in range(4000):
        ae.adam_step(params, {"W": ae.tied_grad(X, params["W"])}, state, lr=1e-2)
    Q, _ = np.linalg.qr(params["W"].T)
    s = np.linalg.svd(basis.T @ Q, compute_uv=False)
    assert s.min() > 1 - 1e-6          # cosines of the principal angles
    z, xh = ae.tied_forward(X, params["W"])
    assert ae.mse(xh, X) < 1e-8


def test_tied_grad_finite_differences():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(6, 9))
    Wt = rng.normal(size=(3, 9))
    gr = ae.tied_grad(X, Wt)
    loss = lambda W: ae.mse(ae.tied_forward(X, W)[1], X)
    for idx in [(0, 0), (1, 4), (2, 8)]:
        Wp, Wm = Wt.copy(), Wt.copy()
        Wp[idx] += 1e-6
        Wm[idx] -= 1e-6
        assert (loss(Wp) - loss(Wm)) / 2e-6 == pytest.approx(gr[idx], rel=1e-6)


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p = {"w": rng.normal(size=(4, 3))}
    tw = torch.tensor(p["w"].copy(), requires_grad=True)
    opt = torch.optim.Adam([tw], lr=1e-3)
    state = {}
    for step in range(5):
        gr = rng.normal(size=(4, 3))
        ae.adam_step(p, {"w": gr}, state, lr=1e-3)
        tw.grad = torch.tensor(gr)
        opt.step()
    assert np.allclose(p["w"], tw.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_norm_stats():
    F = np.random.default_rng(7).random((100, 3, 4))
    F[:, 0, 0] = 2.0                       # constant pixel -> floored std
    mu, sd = ae.norm_stats(F)
    X = F.reshape(100, -1)
    assert np.allclose(mu, X.mean(0))
    assert sd[0] == pytest.approx(1e-12 * X.std(0).max())
    assert np.allclose(sd[1:], X.std(0)[1:])


def test_bf16_rounding_matches_torch_and_ties():
    import torch
    rng = np.random.default_rng(31)
    x = (rng.standard_normal(20000) * 10.0 ** rng.integers(-20, 20, 20000)).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ae.bf16(x), want)
    # exact ties: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7 and goes to the even 1;
    # 1 + 3 * 2^-8 goes up to 1 + 2^-6
    t = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8)], np.float32)
    assert np.array_equal(ae.bf16(t), np.array([1.0, 1 + 2.0 ** -6, -1.0], np.float32))


def test_fma32_is_a_single_rounding():
    """Against exact rational arithmetic: the nearest FP32 value to a b + c (ties to
    even), found among the neighbours of the FP64 result."""
    from fractions import Fraction
    rng = np.random.default_rng(32)
    a, b, c = (rng.standard_normal(3000).astype(np.float32) * np.float32(s) for s in (1.0, 3.0, 0.5))
    # cases where the FP64 sum ties two FP32 values and only the discarded tail decides:
    # a b + c = 1 + 2^-24 + 2^-60 (must round up to 1 + 2^-23, not to the even 1) and
    # 1 + 3 2^-24 - 2^-60 (must round down to 1 + 2^-23, not to the even 1 + 2^-22); and
    # the exact tie 1 + 2^-24 (to the even 1)
    t = 2.0 ** -18
    a = np.concatenate([a, np.float32([-(1 - t) * 2.0 ** -24, (1 - t) * 2.0 ** -24, 1 + 2.0 ** -12])])
    b = np.concatenate([b, np.float32([1 + t, 1 + t, 1 + 2.0 ** -12])])
    c = np.concatenate([c, np.float32([1 + 2.0 ** -23, 1 + 2.0 ** -23, -(2.0 ** -11)])])
    got = ae.fma32(a, b, c)
    assert list(got[-3:]) == [np.float32(1 + 2.0 ** -23), np.float32(1 + 2.0 ** -23), np.float32(1.0)]
    for k in range(len(a)):
        exact = Fraction(float(a[k])) * Fraction(float(b[k])) + Fraction(float(c[k]))
        x0 = np.float32(float(exact))
        cands = [np.nextafter(x0, np.float32(-np.inf)), x0, np.nextafter(x0, np.float32(np.inf))]
        dist = [abs(Fraction(float(v)) - exact) for v in cands]
        best = min(dist)
        ties = [v for v, d in zip(cands, dist) if d == best]
        want = ties[0] if len(ties) == 1 else [v for v in ties if (np.float32(v).view(np.uint32) & 1) == 0][0]
        assert got[k] == want, (k, got[k], want)


def test_bf16_form_is_close_to_the_fp64_model():
    """The BF16 form differs from the FP64 model by about the bfloat16 rounding of its
    operands (2^-9 relative per operand), and equals it when every operand is already a
    bfloat16 value."""
    F = synth.histograms(64, seed=33, dtype=np.float32)
    W = synth.dense_ae_weights()
    mu, sd = ae.norm_stats(F.astype(np.float64))
    mu32, sd32 = mu.astype(np.float32), sd.astype(np.float32)
    rsd32 = (np.float32(1) / sd32).astype(np.float32)
    z16 = ae.dense_encode_bf16(F, mu32, rsd32, W)
    z64 = ae.dense_encode(ae.normalize(F.astype(np.float64), mu, sd), W)
    rel = np.abs(z16 - z64).max() / np.abs(z64).max()
    assert 1e-5 < rel < 2e-2
    # operands already in bfloat16: the form reduces to the exact model on them
    Wb = {k: ae.bf16(np.asarray(v, np.float32)).astype(np.float64) for k, v in W.items()}
    Wb32 = {k: v.astype(np.float32) for k, v in Wb.items()}
    xb = ae.bf16_encode_input(F.reshape(64, -1), mu32, rsd32)
    zb = ae.dense_encode_bf16(F, mu32, rsd32, Wb32)
    assert np.allclose(zb, ae.dense_encode(xb.astype(np.float64), Wb), rtol=1e-12, atol=1e-12)


def test_bf16_training_form():
    """The BF16 training form rounds both operands of every product to bfloat16 (FP32
    master weights, exact products, FP64 sums here).  Pinned against torch's own bfloat16
    conversion: each product, and the whole forward pass written with torch.nn.functional.
    The backward pass has the FP64 pass's structure (pinned by autograd and finite
    differences) and must stay within the bfloat16 operand error of it, without being
    equal to it."""
    import torch
    rng = np.random.default_rng(5)
    A = rng.normal(size=(7, 33)).astype(np.float32)
    B = rng.normal(size=(33, 5)).astype(np.float32)
    bft = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64)
    assert np.allclose(ae._mm(A, B, ae.bf16), (bft(A) @ bft(B)).numpy(), rtol=1e-14, atol=1e-14)
    W = {k: v.astype(np.float32) for k, v in small_weights().items()}
    X = rng.normal(size=(6, 50)).astype(np.float32)
    c = ae.dense_forward_train(X, W, rnd=ae.bf16)
    lin = lambda x, w, b: bft(x.numpy()) @ bft(w).T + torch.from_numpy(W[b]).double()
    h1 = torch.relu(lin(torch.from_numpy(X), W["W1"], "b1"))
    z = lin(h1, W["W2"], "b2")
    h3 = torch.relu(lin(z, W["W3"], "b3"))
    xh = lin(h3, W["W4"], "b4")
    for k, v in (("h1", h1), ("z", z), ("h3", h3), ("xh", xh)):
        assert np.allclose(c[k], v.numpy(), rtol=1e-13, atol=1e-13), k
    W64 = {k: v.astype(np.float64) for k, v in W.items()}
    g64 = ae.dense_backward(ae.dense_forward_train(X.astype(np.float64), W64), W64)
    g16 = ae.dense_backward(c, W, rnd=ae.bf16)
    for k in W:
        rel = np.linalg.norm(g16[k] - g64[k]) / np.linalg.norm(g64[k])
        assert 1e-5 < rel < 3e-2, (k, rel)
