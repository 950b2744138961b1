"""Pins for oracle.predict."""
import numpy as np

from oracle import itergp as oi
from oracle import kernels as ok
from oracle import likelihood as lk
from oracle import newton as on
from oracle import predict as op


def _fit(seed=0, N=8, C=3, j=None, policy="unit"):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, 2))
    Xs = rng.standard_normal((5, 2))
    y = rng.integers(0, C, size=N)
    KX = ok.kernel_matrix(X, X, "rbf", 1.0, 1.3)
    Kf = ok.full_kernel_cn(KX, C)
    F = rng.standard_normal((N, C))
    Wp = lk.softmax_hessian_pinv_blocks(F)
    Khat = Kf + lk.dense_block_diag(Wp)
    rhs = on.pseudo_target_offset(F, y)
    n = N * C
    v, Q, S, T, info = oi.itergp(lambda V: Kf @ V, lambda V: lk.apply_blocks(Wp, V), rhs,
                                 np.zeros((n, 0)), np.zeros((n, 0)), policy=policy,
                                 j_max=n if j is None else j, recycle=False,
                                 tol_abs=0, tol_rel=0)
    return X, Xs, v, Q, Khat, C


def test_full_budget_variance_equals_exact():
    X, Xs, v, Q, Khat, C = _fit()
    got = op.predictive_var_root(Xs, X, Q, C, "rbf", 1.0, 1.3)
    ref = op.predictive_var_exact(Xs, X, Khat, C, "rbf", 1.0, 1.3)
    np.testing.assert_allclose(got, ref, rtol=1e-8, atol=1e-10)
    mean = op.predictive_mean(Xs, X, v, C, "rbf", 1.0, 1.3)
    Ks = np.kron(ok.kernel_matrix(Xs, X, "rbf", 1.0, 1.3), np.eye(C))
    np.testing.assert_allclose(mean.reshape(-1), Ks @ np.linalg.solve(Khat, Khat @ v),
                               rtol=1e-10)


def test_variance_non_increasing_in_j():
    prev = None
    for j in range(0, 25, 3):
        X, Xs, v, Q, Khat, C = _fit(1, j=j, policy="cg")
        var = op.predictive_var_root(Xs, X, Q, C, "rbf", 1.0, 1.3)
        if prev is not None:
            assert np.all(var <= prev + 1e-12)
        assert np.all(var >= -1e-10)
        prev = var


def test_probit_limits():
    rng = np.random.default_rng(2)
    m = rng.standard_normal((6, 4))
    p0 = op.probit_probs(m, np.zeros_like(m))
    np.testing.assert_allclose(p0, lk.softmax(m), rtol=1e-14)
    # growing variance flattens the prediction towards uniform
    p1 = op.probit_probs(m, np.full_like(m, 1e12))
    np.testing.assert_allclose(p1, 0.25, atol=1e-5)
    ent = lambda p: -(p * np.log(p)).sum(1)
    assert np.all(ent(op.probit_probs(m, np.full_like(m, 3.0))) >= ent(p0) - 1e-12)


def test_per_class_predictions_match_dense_definition():
    rng = np.random.default_rng(22)
    X, Xs = rng.standard_normal((25, 2)), rng.standard_normal((7, 2))
    ells, oss = [0.6, 1.4], [0.8, 1.9]
    C = 2
    v = rng.standard_normal(25 * C)
    Q = rng.standard_normal((25 * C, 6))
    Kx = ok.full_kernel_cn_per_class(ok.kernel_matrices_per_class(Xs, X, "rbf", ells, oss))
    Kss = ok.full_kernel_cn_per_class(ok.kernel_matrices_per_class(Xs, Xs, "rbf", ells, oss))
    mean = (Kx @ v).reshape(7, C)
    var = np.diag(Kss - Kx @ Q @ Q.T @ Kx.T).reshape(7, C)
    np.testing.assert_allclose(op.predictive_mean_per_class(Xs, X, v, "rbf", ells, oss), mean,
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(op.predictive_var_root_per_class(Xs, X, Q, "rbf", ells, oss), var,
                               rtol=1e-12, atol=1e-11)


# The probit approximation of the predictive class probabilities (appendix on
# the large-scale experiment) replaces the logistic sigmoid by the Gaussian cdf
# Phi(lam x) whose slope at 0 equals the sigmoid's (1/4), i.e.
# lam = sqrt(2 pi) / 4, and uses the exact Gaussian integral of that cdf:
#     int Phi(lam x) N(x; m, v) dx = Phi(lam m / sqrt(1 + lam^2 v)).
# In the binary case (C = 2, logits [m, 0], variances [v, 0]) the softmax of
# the scaled logits is sigmoid(kappa(v) m), so the scale kappa(v) that
# probit_probs applies can be read back and checked against that integral,
# computed here by adaptive quadrature; the constant lam is derived from
# the slope condition, not taken from the function under test.

def _adaptive_expect(fn, m, v):
    """E[fn(x)] for x ~ N(m, v) by adaptive quadrature (fn may vary on a scale
    much finer than sqrt(v), where Gauss-Hermite is not accurate)."""
    from scipy.integrate import quad
    if v == 0.0:
        return float(fn(np.float64(m)))
    sd = np.sqrt(v)
    dens = lambda x: np.exp(-0.5 * ((x - m) / sd) ** 2) / (sd * np.sqrt(2.0 * np.pi))
    lo, hi = m - 40.0 * sd, m + 40.0 * sd
    pts = sorted({min(max(p, lo), hi) for p in (-10.0, -3.0, 0.0, 3.0, 10.0)})
    val, err = quad(lambda x: fn(x) * dens(x), lo, hi, points=pts, epsabs=1e-14,
                    epsrel=1e-13, limit=400)
    return float(val)


def _binary_probit(m, v):
    return op.probit_probs(np.array([[m, 0.0]]), np.array([[v, 0.0]]))[0, 0]


def test_probit_scale_is_the_exact_gaussian_smoothing_of_the_slope_matched_cdf():
    from scipy.special import logit, ndtr, ndtri
    lam = np.sqrt(2.0 * np.pi) / 4.0                 # Phi'(0) lam = sigmoid'(0) = 1/4
    for v in [0.0, 0.05, 0.3, 1.0, 2.5, 7.0, 30.0, 400.0]:
        for m in [0.4, -1.3, 2.2]:
            kappa = logit(_binary_probit(m, v)) / m
            # the quadrature of the probit-link integral, mapped back to the
            # scale of its argument: Phi(lam m kappa_ref) = E[Phi(lam x)]
            kappa_ref = ndtri(_adaptive_expect(lambda x: ndtr(lam * x), m, v)) / (lam * m)
            assert abs(kappa - kappa_ref) <= 1e-9 * kappa_ref, (m, v, kappa, kappa_ref)


def test_binary_probit_within_its_error_of_the_logistic_normal_integral():
    from scipy.special import expit, ndtr
    lam = np.sqrt(2.0 * np.pi) / 4.0
    # two substitutions of sigmoid by Phi(lam .), each off by at most this much
    t = np.linspace(-30.0, 30.0, 600001)
    sub_err = float(np.abs(expit(t) - ndtr(lam * t)).max())
    assert 0.017 < sub_err < 0.018
    worst = 0.0
    for v in np.concatenate([np.linspace(0.0, 4.0, 21), np.geomspace(4.0, 1e3, 15)]):
        for m in np.linspace(-8.0, 8.0, 41):
            exact = _adaptive_expect(expit, m, v)
            worst = max(worst, abs(_binary_probit(m, v) - exact))
    assert worst <= 2.0 * sub_err
    # measured maximum over this grid for the slope-matched constant: 0.0150
    # (3/pi^2 in place of pi/8 gives 0.023, 8/pi 0.20, no square root 0.27)
    assert worst <= 0.016
