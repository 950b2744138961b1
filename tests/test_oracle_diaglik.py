"""Pins of the oracle's IterNCGP for likelihoods with a diagonal negative
Hessian (Poisson with log link, Gaussian), against facts fixed outside it:

* the textbook Newton update for the Laplace mode,
  f_new = (K^{-1} + W)^{-1} (W f + grad log p(y | f)) (Rasmussen & Williams,
  eq. 3.18), written as K (I + W K)^{-1} (W f + grad);
* the Gaussian posterior mean K (K + s^2 I)^{-1} y, reached in one step;
* the stationarity of the Poisson mode, f = K (y - exp f);
* finite differences of the log likelihoods.
"""
import numpy as np
import pytest

from oracle import itergp as oi
from oracle import kernels as ok
from oracle import likelihood as lk


@pytest.fixture(scope="module")
def pois():
    # moderate counts (log rate sin(6x)), so that full Newton steps from f = 0
    # converge without a line search
    X = np.linspace(0.0, 1.0, 60)[:, None]
    y = np.random.default_rng(8).poisson(np.exp(np.sin(6.0 * X[:, 0])))
    K = ok.kernel_matrix(X, X, "rbf", 0.2, 1.0)
    return X, y, K


def _textbook_newton(K, f, y):
    # (K^{-1} + W)^{-1} = K (I + W K)^{-1}, which avoids inverting K
    lam = np.exp(f)
    W = np.diag(lam)
    grad = y - lam
    return K @ np.linalg.solve(np.eye(len(f)) + W @ K, W @ f + grad)


def test_poisson_full_budget_unit_policy_is_textbook_newton(pois):
    _, y, K = pois
    n = len(y)
    recs = oi.iterncgp_diag(lambda V: K @ V, y, 4, "poisson", policy="unit", j_max=n,
                            recycle=False, tol_abs=0.0, tol_rel=0.0)
    f = np.zeros(n)
    for rec in recs:
        f = _textbook_newton(K, f, y.astype(float))
        assert np.allclose(rec.F[:, 0], f, rtol=1e-6, atol=1e-6 * np.abs(f).max())


def test_poisson_cg_full_budget_equals_unit(pois):
    _, y, K = pois
    n = len(y)
    kw = dict(j_max=n, recycle=False, tol_abs=0.0, tol_rel=0.0)
    a = oi.iterncgp_diag(lambda V: K @ V, y, 3, "poisson", policy="unit", **kw)
    b = oi.iterncgp_diag(lambda V: K @ V, y, 3, "poisson", policy="cg", **kw)
    for ra, rb in zip(a, b):
        assert np.linalg.norm(ra.F - rb.F) <= 1e-6 * np.linalg.norm(ra.F)


def test_poisson_mode_is_stationary(pois):
    _, y, K = pois
    n = len(y)
    recs = oi.iterncgp_diag(lambda V: K @ V, y, 12, "poisson", policy="unit", j_max=n,
                            recycle=False, tol_abs=0.0, tol_rel=0.0)
    f = recs[-1].F[:, 0]
    assert np.linalg.norm(f - K @ (y - np.exp(f))) <= 1e-6 * np.linalg.norm(f)
    assert recs[-1].rel_change < 1e-10


def test_gaussian_one_step_is_posterior_mean():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((60, 2))
    K = ok.kernel_matrix(X, X, "matern32", 0.8, 1.3)
    y = rng.standard_normal(60)
    s2 = 0.3
    recs = oi.iterncgp_diag(lambda V: K @ V, y, 1, "gaussian", noise_var=s2, policy="cg",
                            j_max=60, recycle=False, tol_abs=0.0, tol_rel=0.0)
    ref = K @ np.linalg.solve(K + s2 * np.eye(60), y)
    assert np.linalg.norm(recs[0].F[:, 0] - ref) <= 1e-8 * np.linalg.norm(ref)
    # with recycling, a second step stays at the mode
    recs2 = oi.iterncgp_diag(lambda V: K @ V, y, 2, "gaussian", noise_var=s2, policy="cg",
                             j_max=60, recycle=True, tol_abs=1e-12, tol_rel=0.0)
    assert np.linalg.norm(recs2[1].F[:, 0] - ref) <= 1e-8 * np.linalg.norm(ref)


def test_diag_terms_match_finite_differences():
    rng = np.random.default_rng(5)
    f = rng.normal(size=7)
    y = rng.poisson(2.0, size=7)
    h = 1e-6
    for name, ll in (("poisson", lambda f: lk.poisson_loglik(f, y)),
                     ("gaussian", lambda f: -0.5 * np.sum((y - f) ** 2) / 0.7)):
        grad, wd = oi.diag_likelihood_terms(name, f, y, 0.7)
        E = np.eye(7)
        fd = np.array([(ll(f + h * e) - ll(f - h * e)) / (2 * h) for e in E])
        np.testing.assert_allclose(grad, fd, atol=1e-6)
        g = lambda f: oi.diag_likelihood_terms(name, f, y, 0.7)[0]
        hd = np.array([(g(f + h * e) - g(f - h * e)) / (2 * h) for e in E])
        np.testing.assert_allclose(np.diag(-hd), 1.0 / wd, rtol=1e-6)
