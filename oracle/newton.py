"""QoI-restoring projection with Lagrange multipliers (Section III Stage 5, Eq. 6).

Reading of the Stage-5 problem (the paper calls it a non-linear projection with a convex
distance, linear moment constraints and a dual Newton method):

    f_c = argmin_x  1/2 ||x - ft||^2   subject to  A x = b,  x >= 0

with b the moments of the original histogram and ft the reconstruction.  Its dual
theta(lam) = 1/2 ||x(lam) - ft||^2 + lam^T (A x(lam) - b), x(lam) = max(0, ft - A^T lam),
is concave with gradient g = A x(lam) - b and Hessian -A diag(x > 0) A^T.  Eq. 6 is the
Newton step on it with step size s: lam <- lam + s H^-1 g, H = A diag(x > 0) A^T.

Stopping rule: |g_k| <= 1e-13 * (sum_j |A_kj| x_j + 1e-300) for every k.
Round 1: s = 1, at most 50 updates (Section III Stage 5).
Without positivity (an alternative reading, `project_linear`) the correction is the
orthogonal projection onto {A x = b}, whose multipliers solve (A A^T) lam = A ft - b.  Round 2 (for histograms
round 1 leaves unconverged): from the round-1 multipliers, either Armijo backtracking
on theta (default) or the fixed step s = 0.01, both with at most 400 updates.  A
histogram that still fails is stored verbatim.  A Cholesky pivot <= 1e-14 trace(H)
counts as failure.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid

GTOL = 1e-13
PIVTOL = 1e-14
ARMIJO_C = 1e-4
ARMIJO_HALVINGS = 40


def x_of(ft: np.ndarray, A: np.ndarray, lam: np.ndarray) -> np.ndarray:
    return np.maximum(0.0, ft - A.T @ lam)


def cholesky_solve(Hm: np.ndarray, g: np.ndarray):
    """Solve Hm d = g for a 4x4 SPD matrix; None if a pivot is not clearly positive."""
    n = Hm.shape[0]
    tr = np.trace(Hm)
    Lm = np.zeros_like(Hm)
    for k in range(n):
        piv = Hm[k, k] - np.dot(Lm[k, :k], Lm[k, :k])
        if not (piv > PIVTOL * tr):
            return None
        Lm[k, k] = np.sqrt(piv)
        for i in range(k + 1, n):
            Lm[i, k] = (Hm[i, k] - np.dot(Lm[i, :k], Lm[k, :k])) / Lm[k, k]
    y = np.zeros(n)
    for i in range(n):
        y[i] = (g[i] - np.dot(Lm[i, :i], y[:i])) / Lm[i, i]
    d = np.zeros(n)
    for i in range(n - 1, -1, -1):
        d[i] = (y[i] - np.dot(Lm[i + 1:, i], d[i + 1:])) / Lm[i, i]
    return d


def theta(ft, A, b, lam):
    x = x_of(ft, A, lam)
    return 0.5 * np.dot(x - ft, x - ft) + np.dot(lam, A @ x - b)


def converged(g, A, x):
    sc = np.abs(A) @ x + 1e-300
    return bool(np.all(np.abs(g) <= GTOL * sc))


def newton_round(ft, A, b, lam, s, max_iter, mode):
    """mode: 'fixed' (step s) or 'armijo'. Returns (lam, converged, updates)."""
    lam = np.array(lam, np.float64)
    for it in range(max_iter + 1):
        x = x_of(ft, A, lam)
        g = A @ x - b
        if converged(g, A, x):
            return lam, True, it
        if it == max_iter:
            return lam, False, it
        m = x > 0
        Hm = (A * m) @ A.T
        d = cholesky_solve(Hm, g)
        if d is None:
            return lam, False, it
        if mode == "fixed":
            lam = lam + s * d
        else:
            t0 = theta(ft, A, b, lam)
            gd = float(np.dot(g, d))
            step = 1.0
            for _ in range(ARMIJO_HALVINGS):
                cand = lam + step * d
                if theta(ft, A, b, cand) >= t0 + ARMIJO_C * step * gd:
                    break
                step *= 0.5
            else:
                return lam, False, it
            lam = cand
    return lam, False, max_iter


def scaled_residual(ft, A, b, lam) -> float:
    """max_k |g_k| / (sum_j |A_kj| x_j + 1e-300): the stopping rule's measure."""
    x = x_of(ft, A, lam)
    return float(np.max(np.abs(A @ x - b) / (np.abs(A) @ x + 1e-300)))


def warm_ok(ft, A, b, lam0, s) -> bool:
    """Accept a warm start unless one Newton step from it makes the scaled residual grow."""
    x = x_of(ft, A, lam0)
    g0 = A @ x - b
    if converged(g0, A, x):
        return True
    d = cholesky_solve((A * (x > 0)) @ A.T, g0)
    if d is None:
        return False
    return scaled_residual(ft, A, b, lam0 + s * d) <= scaled_residual(ft, A, b, lam0)


def analytic_start(ft: np.ndarray, b: np.ndarray, g: Grid) -> np.ndarray:
    """The analytic-linear warm start: the multipliers of the projection without the
    positivity constraint, lam0 = (A A^T)^-1 (A ft - b).  Exact whenever no cell of
    ft - A^T lam0 is negative (then it is the Stage-5 solution itself); otherwise Newton
    continues from it under the warm-start acceptance rule of `project`."""
    A = g.A()
    return np.linalg.solve(A @ A.T, A @ np.asarray(ft, np.float64).reshape(-1) - b)


def project_linear(ft: np.ndarray, b: np.ndarray, g: Grid):
    """Reading without positivity: the orthogonal projection of ft onto {A x = b},
    x = ft - A^T lam with (A A^T) lam = A ft - b (the plain definition, one solve)."""
    A = g.A()
    ftv = np.asarray(ft, np.float64).reshape(-1)
    lam = np.linalg.solve(A @ A.T, A @ ftv - b)
    return dict(lam=lam, x=(ftv - A.T @ lam).reshape(np.shape(ft)), status=0, iters=1, warm_rejected=False)


# ---- KL / I-divergence reading of the correction -------------------------------------------
#
#     f_c = argmin_x  sum_j x_j log(x_j / ft_j) - x_j + ft_j   subject to  A x = b
#
# over the cells where ft_j > 0 (the others stay 0).  Stationarity gives the multiplicative
# form x(lam) = ft+ exp(-A^T lam), ft+ = max(ft, 0).  The dual
# D(lam) = -sum_j x_j(lam) - lam^T b is concave with gradient g = A x(lam) - b and Hessian
# -A diag(x) A^T, so the Newton step is lam <- lam + s H^-1 g with H = A diag(x) A^T; the
# stopping rule, rounds and Armijo backtracking (on D) are those of the L2 reading.

def x_kl(ft: np.ndarray, A: np.ndarray, lam: np.ndarray) -> np.ndarray:
    return np.maximum(ft, 0.0) * np.exp(-(A.T @ lam))


def dual_kl(ft, A, b, lam) -> float:
    return -float(np.sum(x_kl(ft, A, lam))) - float(np.dot(lam, b))


def newton_round_kl(ft, A, b, lam, s, max_iter, mode):
    """As newton_round, for the KL reading.  Returns (lam, converged, updates)."""
    lam = np.array(lam, np.float64)
    for it in range(max_iter + 1):
        x = x_kl(ft, A, lam)
        g = A @ x - b
        if converged(g, A, x):
            return lam, True, it
        if it == max_iter:
            return lam, False, it
        d = cholesky_solve((A * x) @ A.T, g)
        if d is None:
            return lam, False, it
        if mode == "fixed":
            lam = lam + s * d
        else:
            t0 = dual_kl(ft, A, b, lam)
            gd = float(np.dot(g, d))
            step = 1.0
            for _ in range(ARMIJO_HALVINGS):
                cand = lam + step * d
                if dual_kl(ft, A, b, cand) >= t0 + ARMIJO_C * step * gd:
                    break
                step *= 0.5
            else:
                return lam, False, it
            lam = cand
    return lam, False, max_iter


def project_kl(ft: np.ndarray, b: np.ndarray, g: Grid, s: float = 1.0, max_iter: int = 50,
               max_iter2: int = 400, fallback: str = "backtrack"):
    """KL reading: dict(lam, x, status, iters, warm_rejected) as project()."""
    A = g.A()
    ftv = np.asarray(ft, np.float64).reshape(-1)
    lam1, ok, it1 = newton_round_kl(ftv, A, b, np.zeros(4), s, max_iter, "fixed")
    if ok:
        return dict(lam=lam1, x=x_kl(ftv, A, lam1).reshape(np.shape(ft)), status=0, iters=it1, warm_rejected=False)
    mode = "fixed" if fallback == "paper" else "armijo"
    lam2, ok2, it2 = newton_round_kl(ftv, A, b, lam1, 0.01 if fallback == "paper" else 1.0, max_iter2, mode)
    if ok2:
        return dict(lam=lam2, x=x_kl(ftv, A, lam2).reshape(np.shape(ft)), status=1, iters=it1 + it2,
                    warm_rejected=False)
    return dict(lam=np.zeros(4), x=None, status=2, iters=it1 + it2, warm_rejected=False)


def project(ft: np.ndarray, b: np.ndarray, g: Grid, s: float = 1.0, max_iter: int = 50,
            max_iter2: int = 400, fallback: str = "backtrack", lam0=None, positivity: bool = True):
    """Project one reconstruction ft (n_perp, n_par) onto {A x = b, x >= 0}.

    lam0: optional warm start; rejected (cold start, flag 'warm_rejected') if its first
    Newton step makes the scaled residual grow (or if round 1 allows no update).  Returns dict(lam, x, status, iters,
    warm_rejected): status 0 = round 1 converged, 1 = round 2 converged, 2 = failed
    (store verbatim).
    """
    if not positivity:
        return project_linear(ft, b, g)
    A = g.A()
    ftv = np.asarray(ft, np.float64).reshape(-1)
    rejected = False
    lam = np.zeros(4)
    if lam0 is not None:
        lam0 = np.asarray(lam0, np.float64)
        if max_iter >= 1 and np.all(np.isfinite(lam0)) and warm_ok(ftv, A, b, lam0, s):
            lam = lam0
        else:
            rejected = True
    res = _project_from(ftv, A, b, ft.shape, lam, s, max_iter, max_iter2, fallback)
    res["warm_rejected"] = rejected
    return res


def _project_from(ftv, A, b, shape, lam, s, max_iter, max_iter2, fallback):
    ft = ftv.reshape(shape)
    lam1, ok, it1 = newton_round(ftv, A, b, lam, s, max_iter, "fixed")
    if ok:
        return dict(lam=lam1, x=x_of(ftv, A, lam1).reshape(ft.shape), status=0, iters=it1)
    mode = "fixed" if fallback == "paper" else "armijo"
    s2 = 0.01 if fallback == "paper" else 1.0
    lam2, ok2, it2 = newton_round(ftv, A, b, lam1, s2, max_iter2, mode)
    if ok2:
        return dict(lam=lam2, x=x_of(ftv, A, lam2).reshape(ft.shape), status=1, iters=it1 + it2)
    return dict(lam=np.zeros(4), x=None, status=2, iters=it1 + it2)


def apply(ft: np.ndarray, lam: np.ndarray, g: Grid, positivity: bool = True, kl: bool = False) -> np.ndarray:
    """Decompression-side correction f_c = max(0, ft - A^T lam) (or ft - A^T lam without
    positivity, or max(ft, 0) exp(-A^T lam) in the KL reading) for one histogram."""
    ftv = np.asarray(ft, np.float64).reshape(-1)
    lam = np.asarray(lam, np.float64)
    if kl:
        return x_kl(ftv, g.A(), lam).reshape(ft.shape)
    if not positivity:
        return (ftv - g.A().T @ lam).reshape(ft.shape)
    return x_of(ftv, g.A(), lam).reshape(ft.shape)


def project_bruteforce(ft: np.ndarray, b: np.ndarray, g: Grid):
    """Exact KKT point by enumerating every active set (tiny grids only).

    For each set Z of cells fixed at zero, solve the equality-constrained projection on
    the free cells and keep the candidate that is primal feasible (x >= 0) and dual
    feasible (the multipliers of x >= 0 are >= 0).
    """
    A = g.A()
    f = np.asarray(ft, np.float64).reshape(-1)
    N = f.size
    best = None
    for mask in range(1 << N):
        free = np.array([(mask >> k) & 1 == 0 for k in range(N)])
        Af = A[:, free]
        M = Af @ Af.T
        if np.linalg.matrix_rank(M) < 4:
            continue
        lam = np.linalg.solve(M, Af @ f[free] - b)
        x = np.zeros(N)
        x[free] = f[free] - Af.T @ lam
        if np.any(x[free] < -1e-12):
            continue
        mu = -(f[~free] - A[:, ~free].T @ lam)     # multipliers of x >= 0 on the fixed set
        if np.any(mu < -1e-12):
            continue
        cand = (np.linalg.norm(x - f), x, lam)
        if best is None or cand[0] < best[0]:
            best = cand
    return None if best is None else dict(x=best[1].reshape(ft.shape), lam=best[2])
