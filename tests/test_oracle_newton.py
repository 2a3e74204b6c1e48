"""Pins of the oracle's Lagrange/Newton projection (Section III Stage 5, Eq. 6)."""
import numpy as np
import pytest

from oracle import grid, moments, newton
from paper_2212_10733_amd import synth


def positive_case(seed=0, n=39, rel=1e-3):
    g = grid.make_grid(n, n)
    rng = np.random.default_rng(seed)
    jj, ii = np.meshgrid(np.linspace(0, 1, n), np.linspace(0, 1, n), indexing="ij")
    f = 1.0 + np.exp(-((ii - 0.4) ** 2 + (jj - 0.3) ** 2) * 4) + 0.1 * rng.random((n, n))
    ft = f + rel * rng.normal(size=f.shape)
    return g, f, ft


def test_closed_form_without_active_positivity():
    # All cells stay positive, so the projection is the least-norm correction onto A x = b.
    g, f, ft = positive_case()
    A = g.A()
    b = moments.moments(f, g)
    res = newton.project(ft, b, g)
    lam_cf = np.linalg.solve(A @ A.T, A @ ft.ravel() - b)
    assert res["status"] == 0 and res["iters"] <= 2
    assert np.allclose(res["lam"], lam_cf, rtol=1e-9, atol=1e-12 * np.abs(lam_cf).max())
    assert np.allclose(res["x"].ravel(), ft.ravel() - A.T @ lam_cf, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_bruteforce_active_sets_on_3x3(seed):
    g = grid.make_grid(3, 3)
    rng = np.random.default_rng(seed)
    f = rng.random((3, 3)) + 0.2
    f[rng.integers(0, 3), rng.integers(0, 3)] = 0.0
    ft = f + 0.3 * rng.normal(size=(3, 3))       # large enough that cells hit zero
    b = moments.moments(f, g)
    ref = newton.project_bruteforce(ft, b, g)
    res = newton.project(ft, b, g)
    assert ref is not None and res["status"] in (0, 1)
    assert np.allclose(res["x"], ref["x"], atol=1e-12 * np.abs(f).max())


def test_kkt_constraints_nonexpansive_on_synthetic():
    g = grid.make_grid()
    F = synth.histograms(12, seed=11, dtype=np.float64)
    rng = np.random.default_rng(3)
    active = 0
    for f in F:
        ft = f + 0.01 * f.max() * rng.normal(size=f.shape)
        b = moments.moments(f, g)
        res = newton.project(ft, b, g)
        assert res["status"] == 0
        x = res["x"]
        assert np.all(x >= 0)
        assert np.allclose(moments.moments(x, g), b, rtol=1e-13, atol=1e-13 * abs(b[0]))
        assert np.linalg.norm(x - f) <= np.linalg.norm(ft - f) * (1 + 1e-12)
        active += int((x == 0).sum())
    assert active > 0          # positivity was active somewhere


def test_exact_input_needs_no_update_and_scaling():
    g = grid.make_grid()
    f = synth.histograms(1, seed=12, dtype=np.float64)[0]
    b = moments.moments(f, g)
    res = newton.project(f, b, g)
    assert res["iters"] == 0 and np.all(res["lam"] == 0)
    g2, f2, ft2 = positive_case(seed=4)
    b2 = moments.moments(f2, g2)
    r1 = newton.project(ft2, b2, g2)
    r2 = newton.project(7.0 * ft2, 7.0 * b2, g2)
    assert np.allclose(r2["lam"], 7.0 * r1["lam"], rtol=1e-9, atol=1e-12)


def test_mirror_symmetric_input_gives_zero_flow_multiplier():
    g = grid.make_grid(39, 39)
    rng = np.random.default_rng(5)
    half = rng.random((39, 20)) + 0.5
    f = np.concatenate([half, half[:, :19][:, ::-1]], axis=1)
    pert = rng.normal(size=(39, 20))
    ft = f + 0.05 * np.concatenate([pert, pert[:, :19][:, ::-1]], axis=1)
    res = newton.project(ft, moments.moments(f, g), g)
    assert abs(res["lam"][1]) <= 1e-10 * np.abs(res["lam"]).max()


def test_singular_hessian_fails_to_verbatim():
    g = grid.make_grid(5, 5)
    f = np.zeros((5, 5))
    f[2, 2] = 1.0
    ft = np.zeros((5, 5))
    ft[1, 3] = 1.0                      # only one live cell: rank-1 Hessian
    res = newton.project(ft, moments.moments(f, g), g)
    assert res["status"] == 2


def test_paper_fallback_schedule_selectable():
    g, f, ft = positive_case(seed=6, rel=0.05)
    b = moments.moments(f, g)
    r0 = newton.project(ft, b, g, max_iter=0, fallback="paper", max_iter2=3000)
    assert r0["status"] == 1                      # 0.99^k decay still gets there given enough steps
    r1 = newton.project(ft, b, g, max_iter=0, max_iter2=0)
    assert r1["status"] == 2


def test_lambda_precision_magnitudes():
    # FP64 multipliers restore the QoIs to ~1e-13; storing them in FP32 costs ~1e-8 (Section I).
    g = grid.make_grid()
    F = synth.histograms(8, seed=13, dtype=np.float64)
    rng = np.random.default_rng(7)
    e64, e32 = [], []
    for f in F:
        ft = np.maximum(0, f + 3e-3 * f.max() * rng.normal(size=f.shape))
        b = moments.moments(f, g)
        res = newton.project(ft, b, g)
        q = moments.qoi_from_moments(b, g)
        e64.append(moments.qoi_rel_error(q, moments.qoi(newton.apply(ft, res["lam"], g), g), g).max())
        lam32 = res["lam"].astype(np.float32).astype(np.float64)
        e32.append(moments.qoi_rel_error(q, moments.qoi(newton.apply(ft, lam32, g), g), g).max())
    assert max(e64) < 1e-12
    assert 1e-11 < np.median(e32) < 1e-5


def test_warm_start_rules():
    g, f, ft = positive_case(seed=8, rel=0.02)
    b = moments.moments(f, g)
    cold = newton.project(ft, b, g)
    exact = newton.project(ft, b, g, lam0=cold["lam"])
    assert exact["iters"] == 0 and not exact["warm_rejected"]
    near = newton.project(ft, b, g, lam0=cold["lam"] * (1 + 1e-3))
    assert not near["warm_rejected"] and near["iters"] <= cold["iters"]
    assert np.allclose(near["x"], cold["x"], rtol=1e-12, atol=1e-14)
    bad = newton.project(ft, b, g, lam0=np.array([1e6, 0.0, 0.0, 0.0]))   # every cell clipped
    assert bad["warm_rejected"]
    assert np.allclose(bad["lam"], cold["lam"]) and bad["iters"] == cold["iters"]
    nan = newton.project(ft, b, g, lam0=np.array([np.nan, 0, 0, 0]))
    assert nan["warm_rejected"] and nan["iters"] == cold["iters"]


def test_analytic_start():
    """The analytic-linear start (A A^T)^-1 (A ft - b): with no active positivity constraint
    it is the solution itself (0 updates, the least-norm closed form solved independently
    by least squares on the constraint system); it scales with (f, ft); on histograms whose
    tails clip it reaches the same unique projection as the cold start; and the pipeline
    applies it per histogram."""
    g, f, ft = positive_case(seed=9)
    A = g.A()
    b = moments.moments(f, g)
    lam0 = newton.analytic_start(ft, b, g)
    # least-norm correction: the minimum-norm solution of A^T lam ~ (ft - x) with A x = b is
    # the lstsq solution of A^T lam = ft - x*, x* = ft - A^T lam; check it via the normal
    # equations' alternative route, an SVD of A
    U, S, Vt = np.linalg.svd(A, full_matrices=False)
    lam_svd = U @ ((U.T @ (A @ ft.ravel() - b)) / S ** 2)
    assert np.allclose(lam0, lam_svd, rtol=1e-10, atol=1e-13 * np.abs(lam_svd).max())
    res = newton.project(ft, b, g, lam0=lam0)
    assert res["iters"] == 0 and not res["warm_rejected"]
    assert np.allclose(moments.moments(res["x"], g), b, rtol=1e-13)
    assert np.allclose(newton.analytic_start(3.0 * ft, 3.0 * b, g), 3.0 * lam0, rtol=1e-12)
    G = grid.make_grid()
    F = synth.histograms(6, seed=12, dtype=np.float64)
    rng = np.random.default_rng(12)
    clipped = 0
    for fh in F:
        fth = fh + 0.01 * fh.max() * rng.normal(size=fh.shape)
        bh = moments.moments(fh, G)
        cold = newton.project(fth, bh, G)
        warm = newton.project(fth, bh, G, lam0=newton.analytic_start(fth, bh, G))
        assert cold["status"] == 0 and warm["status"] == 0
        assert np.allclose(warm["x"], cold["x"], rtol=0, atol=1e-12 * fh.max())
        clipped += int((cold["x"] == 0).sum())
    assert clipped > 0
    from oracle import pipeline
    Fs = synth.histograms(4, seed=13, dtype=np.float64)
    pc = pipeline.compress(Fs, G, None, None, pipeline.Params(tau=1e-2))
    pa = pipeline.compress(Fs, G, None, None, pipeline.Params(tau=1e-2, analytic_start=True))
    assert pc["stream"] == pa["stream"] and np.array_equal(pc["kstar"], pa["kstar"])
    assert np.allclose(pa["fc"], pc["fc"], rtol=0, atol=1e-12 * Fs.max())
    with pytest.raises(ValueError):
        pipeline.compress(Fs, G, None, None, pipeline.Params(tau=1e-2, analytic_start=True, positivity=False))


def test_mlp_backward_matches_autograd():
    import torch
    from oracle import mlp
    from paper_2212_10733_amd import synth
    P = {k: v.astype(np.float64) for k, v in synth.mlp_weights().items()}
    rng = np.random.default_rng(3)
    for k in ("b1", "b2", "b3"):
        P[k] = rng.normal(0, 0.1, P[k].shape)
    Z = rng.normal(size=(20, 16))
    T = rng.normal(size=(20, 4))
    g = mlp.backward(mlp.forward(Z, P), T, P)
    t = {k: torch.tensor(v, requires_grad=True) for k, v in P.items()}
    z = torch.tensor(Z)
    h = torch.relu(z @ t["W1"].T + t["b1"])
    h = torch.relu(h @ t["W2"].T + t["b2"])
    out = h @ t["W3"].T + t["b3"]
    ((out - torch.tensor(T)) ** 2).mean().backward()
    for k in P:
        assert np.allclose(g[k], t[k].grad.numpy(), rtol=1e-10, atol=1e-12)
    assert synth.mlp_weights()["W1"].shape == (64, 16)
    assert sum(v.size for v in synth.mlp_weights().values()) == 5508


def test_projection_without_positivity():
    """project_linear: A x = b, x - ft orthogonal to the null space of A (an SVD basis,
    not the normal equations the oracle solves), negative values kept, and equal to the
    Stage-5 projection when no cell reaches zero."""
    g = grid.make_grid()
    F = synth.histograms(4, seed=21, dtype=np.float64)
    rng = np.random.default_rng(22)
    A = g.A()
    _, _, Vt = np.linalg.svd(A)
    Z = Vt[4:].T                                  # orthonormal basis of null(A)
    for f in F:
        ft = f + 0.05 * f.max() * rng.normal(size=f.shape)     # plenty of negative cells
        b = moments.moments(f, g)
        res = newton.project_linear(ft, b, g)
        x = res["x"].reshape(-1)
        assert np.allclose(A @ x, b, rtol=1e-12, atol=1e-14 * np.abs(b).max())
        assert np.abs(Z.T @ (x - ft.reshape(-1))).max() < 1e-12 * np.abs(ft).max()
        assert (x < 0).any()
        assert np.allclose(newton.apply(ft, res["lam"], g, positivity=False), res["x"], rtol=0, atol=1e-15)
    g, f, ft = positive_case(seed=23)
    b = moments.moments(f, g)
    lin = newton.project_linear(ft, b, g)
    pos = newton.project(ft, b, g)
    assert np.all(lin["x"] > 0)
    assert np.allclose(lin["lam"], pos["lam"], rtol=1e-10, atol=1e-14)


def test_kl_reading_recovers_a_planted_solution():
    """Plant the answer: for any f >= 0 and lam*, ft = f exp(+A^T lam*) projects (KL) onto
    {A x = A f} at x = f with multipliers lam* (x = ft exp(-A^T lam) satisfies the
    constraints at lam = lam*, and the minimiser is unique)."""
    g = grid.make_grid()
    A = g.A()
    rng = np.random.default_rng(70)
    for s in range(4):
        f = synth.histograms(1, seed=70 + s, dtype=np.float64)[0].reshape(-1)
        lam_star = rng.normal(0, 0.05, 4) / np.abs(A).max(axis=1)
        ft = f * np.exp(A.T @ lam_star)
        res = newton.project_kl(ft.reshape(39, 39), A @ f, g)
        assert res["status"] == 0
        assert np.allclose(res["lam"], lam_star, rtol=1e-9, atol=1e-12 * np.abs(lam_star).max())
        assert np.allclose(res["x"].reshape(-1), f, rtol=1e-10, atol=1e-13 * f.max())
        assert np.array_equal(res["x"].reshape(-1) == 0, f == 0)     # support is kept


def test_kl_reading_matches_a_general_solver_on_3x3():
    """The KL projection on a 3 x 3 grid against SLSQP minimising the I-divergence under
    the four moment constraints (a library optimiser on the plain definition)."""
    from scipy.optimize import minimize
    g = grid.make_grid(3, 3)
    A = g.A()
    rng = np.random.default_rng(71)
    for _ in range(3):
        f = rng.uniform(0.2, 1.0, 9)
        ft = f * rng.uniform(0.9, 1.1, 9)
        b = A @ f
        res = newton.project_kl(ft.reshape(3, 3), b, g)
        assert res["status"] == 0
        obj = lambda x: float(np.sum(x * np.log(x / ft) - x + ft))
        jac = lambda x: np.log(x / ft)
        sol = minimize(obj, ft, jac=jac, method="SLSQP", bounds=[(1e-12, None)] * 9,
                       constraints=[dict(type="eq", fun=lambda x: A @ x - b, jac=lambda x: A)],
                       options=dict(ftol=1e-15, maxiter=500))
        assert sol.success
        assert np.allclose(res["x"].reshape(-1), sol.x, rtol=1e-6, atol=1e-9)
        assert np.allclose(A @ res["x"].reshape(-1), b, rtol=1e-13, atol=1e-15)


def test_kl_pipeline_keeps_the_bound_and_qois():
    """KL where it keeps the bound (flag bit 5), the L2 projection elsewhere: the bound,
    the QoIs and non-negativity hold on every histogram."""
    from oracle import pipeline
    g = grid.make_grid()
    F = synth.histograms(16, seed=72, dtype=np.float64)
    p = pipeline.Params(tau=1e-2, kl=True)
    comp = pipeline.compress(F, g, None, None, p)
    raw = (comp["flags"] & pipeline.FLAG_RAW) != 0
    kl = (comp["flags"] & pipeline.FLAG_KL) != 0
    assert not raw.any() and 0 < kl.sum() < 16
    out = pipeline.decompress(comp, g, None, None, 16, np.float64)
    assert np.allclose(out, comp["fc"], rtol=1e-15, atol=0)
    th = pipeline.tau_h(F, p)
    dist = np.sqrt(((out - F) ** 2).reshape(16, -1).sum(1))
    assert np.all(dist[~raw] <= th[~raw])
    assert np.all(out >= 0)
    err = moments.qoi_rel_error(moments.qoi(F, g), moments.qoi(out, g), g)[~raw]
    assert err.max() < 1e-11
