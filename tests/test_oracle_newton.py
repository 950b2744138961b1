"""Pins for oracle.newton: textbook Newton, mode fixed point, optimiser,
monotone log posterior, Gaussian-likelihood theorem."""
import numpy as np
import scipy.optimize as so

from oracle import kernels as ok
from oracle import likelihood as lk
from oracle import newton as on


def _setup(seed=0, N=10, C=3, D=2, kind="matern32", ell=1.0, os_=2.0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, D))
    y = rng.integers(0, C, size=N)
    KX = ok.kernel_matrix(X, X, kind, ell, os_)
    return KX, ok.full_kernel_cn(KX, C), y, C


def test_step_equals_textbook_newton_step():
    KX, Kf, y, C = _setup()
    F = np.zeros((len(y), C))
    for _ in range(4):
        F_pt, _, _ = on.exact_step(Kf, F, y)
        F_tb = on.textbook_newton_step(Kf, F, y)
        np.testing.assert_allclose(F_pt, F_tb, rtol=1e-8, atol=1e-10)
        F = F_pt


def test_converges_to_mode_fixed_point():
    # at the mode grad Psi = 0, i.e. f* = K grad log p(y | f*)
    KX, Kf, y, C = _setup(1)
    Fs, _ = on.exact_newton(Kf, y, C, 25)
    F = Fs[-1]
    np.testing.assert_allclose(F.reshape(-1), Kf @ lk.softmax_grad(F, y).reshape(-1),
                               atol=1e-10)


def test_log_posterior_increases_and_matches_optimiser():
    KX, Kf, y, C = _setup(2, N=6)
    Fs, vs = on.exact_newton(Kf, y, C, 12)
    psis = [on.log_posterior(Kf, F, y) for F in Fs]
    assert all(b >= a - 1e-12 for a, b in zip(psis, psis[1:]))
    # psi via g^T v equals psi via K^{-1}
    for F, v in zip(Fs[1:], vs):
        assert abs(on.psi_from_v(F, y, v) - on.log_posterior(Kf, F, y)) < 1e-9
    Kinv = np.linalg.inv(Kf)

    def negpsi(f):
        F = f.reshape(-1, C)
        return -(lk.softmax_loglik(F, y) - 0.5 * f @ Kinv @ f)

    def grad(f):
        F = f.reshape(-1, C)
        return -(lk.softmax_grad(F, y).reshape(-1) - Kinv @ f)

    res = so.minimize(negpsi, np.zeros(Kf.shape[0]), jac=grad, method="BFGS",
                      options={"gtol": 1e-11, "maxiter": 10000})
    np.testing.assert_allclose(Fs[-1].reshape(-1), res.x, atol=1e-5)


def test_gaussian_likelihood_converges_in_one_step():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((15, 2))
    K = ok.kernel_matrix(X, X, "rbf", 0.8, 1.5)
    yv = rng.standard_normal(15)
    lam = rng.uniform(0.1, 0.5, size=15)
    f0 = rng.standard_normal(15)           # any start

    def gstep(f):
        grad = (yv - f) / lam               # gradient of log N(y; f, diag(lam))
        return on.exact_step_diag(K, f, grad, lam)

    f1, _, rhs = gstep(f0)
    np.testing.assert_allclose(rhs, yv, rtol=1e-12)        # pseudo-targets = y
    f2, _, _ = gstep(f1)
    np.testing.assert_allclose(f2, f1, rtol=1e-10, atol=1e-12)
    # equals the posterior mean of GP regression (K^{-1} + Lam^{-1})^{-1} Lam^{-1} y
    ref = np.linalg.solve(np.linalg.inv(K) + np.diag(1 / lam), yv / lam)
    np.testing.assert_allclose(f1, ref, rtol=1e-8)


def test_pseudo_target_offset_has_zero_class_sums_beyond_f():
    KX, Kf, y, C = _setup(4)
    rng = np.random.default_rng(5)
    F = rng.standard_normal((len(y), C))
    off = on.pseudo_target_offset(F, y).reshape(-1, C) - F
    np.testing.assert_allclose(off.sum(axis=1), 0.0, atol=1e-12)
