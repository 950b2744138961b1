"""Pins for oracle.itergp.iterncgp_block (Algorithm 1 for a likelihood given
as per-point gradients and C x C negative-Hessian blocks) against facts fixed
independently of it:

* correlated Gaussian observations (log p = -(y_n - f_n)^T Sigma^{-1}
  (y_n - f_n) / 2 per point) make one exact Newton step from f_0 = 0 the GP
  regression posterior mean K (K + I (x) Sigma)^{-1} y, written out densely;
* for a non-quadratic likelihood (softmax plus a ridge on f, so that every
  block is positive definite) each full-budget step equals the Newton step
  f_{i+1} = K (K + W^{-1})^{-1} (f_i + W^{-1} grad), solved densely;
* with C = 1 and the Poisson terms as 1 x 1 blocks it reproduces
  iterncgp_diag (the diagonal form, pinned on its own);
* with CG actions it reaches the same iterate as the dense Newton step when the
  budget is the full dimension.
"""
import numpy as np

from oracle import itergp as oi
from oracle import kernels as ok
from oracle import likelihood as lk


def _gp(seed, N, C, D=2, kind="matern32"):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, D))
    KX = ok.kernel_matrix(X, X, kind, 1.0, 1.0)
    return rng, ok.full_kernel_cn(KX, C)


def _spd_blocks(rng, N, C, floor=0.3):
    A = rng.standard_normal((N, C, C))
    return np.einsum("nij,nkj->nik", A, A) / C + floor * np.eye(C)


def test_correlated_gaussian_one_step_is_regression():
    N, C = 12, 3
    rng, Kf = _gp(0, N, C)
    Sigma = _spd_blocks(rng, N, C)                       # per-point noise covariances
    P = np.linalg.inv(Sigma)                             # W_n = Sigma_n^{-1}
    y = rng.standard_normal((N, C))
    terms = lambda F: (np.einsum("nij,nj->ni", P, y - F), P)
    n = N * C
    rec = oi.iterncgp_block(lambda V: Kf @ V, terms, N, C, 1, policy="unit", j_max=n,
                            recycle=False, tol_abs=0, tol_rel=0)[0]
    noise = lk.dense_block_diag(Sigma)
    mean = Kf @ np.linalg.solve(Kf + noise, y.reshape(-1))
    np.testing.assert_allclose(rec.F.reshape(-1), mean, rtol=1e-9, atol=1e-10)
    # the pseudo-targets of the first step are y itself
    np.testing.assert_allclose(rec.rhs, y.reshape(-1), rtol=1e-12, atol=1e-12)


def _softmax_ridge(y, C, delta):
    def terms(F):
        pi = lk.softmax(F)
        grad = lk.onehot(y, C) - pi - delta * F
        W = np.einsum("ni,ij->nij", pi, np.eye(C)) - np.einsum("ni,nj->nij", pi, pi)
        return grad, W + delta * np.eye(C)
    return terms


def test_full_budget_steps_are_dense_newton_steps():
    N, C = 10, 3
    rng, Kf = _gp(1, N, C)
    y = rng.integers(0, C, size=N)
    terms = _softmax_ridge(y, C, 0.5)
    n = N * C
    recs = oi.iterncgp_block(lambda V: Kf @ V, terms, N, C, 3, policy="unit", j_max=n,
                             recycle=False, tol_abs=0, tol_rel=0)
    F = np.zeros((N, C))
    for rec in recs:
        g, W = terms(F)
        Winv = lk.dense_block_diag(np.linalg.inv(W))
        F = (Kf @ np.linalg.solve(Kf + Winv, F.reshape(-1) + Winv @ g.reshape(-1))).reshape(N, C)
        np.testing.assert_allclose(rec.F, F, rtol=1e-9, atol=1e-10)


def test_cg_full_budget_reaches_the_newton_step():
    N, C = 9, 2
    rng, Kf = _gp(2, N, C)
    y = rng.integers(0, C, size=N)
    terms = _softmax_ridge(y, C, 0.3)
    n = N * C
    rec = oi.iterncgp_block(lambda V: Kf @ V, terms, N, C, 1, policy="cg", j_max=n,
                            recycle=False, tol_abs=0, tol_rel=0)[0]
    g, W = terms(np.zeros((N, C)))
    Winv = lk.dense_block_diag(np.linalg.inv(W))
    F1 = Kf @ np.linalg.solve(Kf + Winv, Winv @ g.reshape(-1))
    np.testing.assert_allclose(rec.F.reshape(-1), F1, rtol=1e-7, atol=1e-9)


def test_poisson_as_blocks_matches_the_diagonal_form():
    N = 15
    rng, Kf = _gp(3, N, 1)
    y = rng.poisson(2.0, size=N).astype(np.float64)
    terms = lambda F: (lk.poisson_grad(F[:, 0], y)[:, None],
                       np.exp(F[:, 0])[:, None, None])
    kw = dict(policy="cg", j_max=8, rank_limit=5, recycle=True, tol_abs=1e-9, tol_rel=1e-9)
    blk = oi.iterncgp_block(lambda V: Kf @ V, terms, N, 1, 3, **kw)
    dia = oi.iterncgp_diag(lambda V: Kf @ V, y, 3, "poisson", **kw)
    for a, b in zip(blk, dia):
        assert a.info.iters == b.info.iters
        np.testing.assert_allclose(a.F, b.F, rtol=1e-12, atol=1e-12)
