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
