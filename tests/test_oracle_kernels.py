"""Pins for oracle.kernels against definitions independent of its code."""
import math

import numpy as np
import pytest
from scipy.special import gamma, kv
from scipy.stats import norm

from oracle import kernels as ok

NU = {"matern12": 0.5, "matern32": 1.5, "matern52": 2.5}


def matern_bessel(r, nu, os_):
    """General Matern covariance via the modified Bessel function K_nu."""
    r = np.asarray(r, dtype=np.float64)
    out = np.full_like(r, os_)
    m = r > 0
    z = math.sqrt(2.0 * nu) * r[m]
    out[m] = os_ * (2.0 ** (1.0 - nu) / gamma(nu)) * z ** nu * kv(nu, z)
    return out


@pytest.mark.parametrize("kind", ["matern12", "matern32", "matern52"])
def test_matern_matches_bessel_definition(kind):
    r = np.concatenate([[0.0], np.geomspace(1e-4, 30.0, 200)])
    got = ok.kernel_of_r2(r * r, kind, 0.7)
    ref = matern_bessel(r, NU[kind], 0.7)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-300)


def test_rbf_matches_gaussian_density_ratio():
    r = np.linspace(0.0, 8.0, 101)
    got = ok.kernel_of_r2(r * r, "rbf", 2.5)
    ref = 2.5 * norm.pdf(r) / norm.pdf(0.0)
    np.testing.assert_allclose(got, ref, rtol=1e-12)


@pytest.mark.parametrize("kind", ok.KINDS)
def test_kernel_matrix_brute_force(kind):
    rng = np.random.default_rng(0)
    X1, X2 = rng.standard_normal((6, 3)), rng.standard_normal((5, 3))
    ell, os_ = 1.3, 0.8
    K = ok.kernel_matrix(X1, X2, kind, ell, os_)
    for i in range(6):
        for j in range(5):
            r = math.dist(X1[i], X2[j]) / ell
            if kind == "rbf":
                ref = os_ * norm.pdf(r) / norm.pdf(0.0)
            else:
                ref = matern_bessel(np.array([r]), NU[kind], os_)[0]
            assert abs(K[i, j] - ref) <= 1e-12 * os_


@pytest.mark.parametrize("kind", ok.KINDS)
def test_kernel_matrix_symmetric_psd_diag(kind):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((40, 4))
    K = ok.kernel_matrix(X, X, kind, 0.9, 1.7)
    assert np.array_equal(K, K.T)
    assert np.all(np.diag(K) == 1.7)
    lam = np.linalg.eigvalsh(K)
    assert lam.min() >= -40 * np.finfo(float).eps * lam.max()


def test_rbf_is_product_of_coordinate_kernels():
    # exp(-|x-y|^2/2l^2) factorises over coordinates; a formula using r
    # instead of r^2 (or a wrong constant) does not.
    rng = np.random.default_rng(2)
    X1, X2 = rng.standard_normal((4, 3)), rng.standard_normal((5, 3))
    K = ok.kernel_matrix(X1, X2, "rbf", 0.6, 1.0)
    P = np.ones((4, 5))
    for d in range(3):
        P *= ok.kernel_matrix(X1[:, d:d + 1], X2[:, d:d + 1], "rbf", 0.6, 1.0)
    np.testing.assert_allclose(K, P, rtol=1e-13)


def test_kernel_matvec_blockwise_equals_dense():
    rng = np.random.default_rng(3)
    X1, X2 = rng.standard_normal((37, 5)), rng.standard_normal((29, 5))
    V = rng.standard_normal((29, 7))
    got = ok.kernel_matvec(X1, X2, V, "matern32", 1.1, 0.5, block=8)
    ref = ok.kernel_matrix(X1, X2, "matern32", 1.1, 0.5) @ V
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_full_kernel_cn_ordering():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((4, 2))
    KX = ok.kernel_matrix(X, X, "rbf", 1.0, 1.0)
    C = 3
    Kf = ok.full_kernel_cn(KX, C)
    for n in range(4):
        for m in range(4):
            for c in range(C):
                for c2 in range(C):
                    assert Kf[n * C + c, m * C + c2] == (KX[n, m] if c == c2 else 0.0)
    v = rng.standard_normal(12)
    np.testing.assert_allclose(ok.apply_full_kernel_cn(KX, v, C), Kf @ v, rtol=1e-14)


def test_per_class_kernels_dense_definition_and_shared_limit():
    """One kernel per latent function: the matrix-free apply equals the dense
    block-diagonal (in NC-ordering) matrix re-indexed to CN-ordering, that
    matrix is symmetric PSD with the class variances on its diagonal, and equal
    hyperparameters reduce to the shared-kernel Kronecker form."""
    rng = np.random.default_rng(21)
    X = rng.standard_normal((30, 3))
    ells, oss = [0.7, 1.3, 2.1], [0.5, 1.0, 1.7]
    Ks = ok.kernel_matrices_per_class(X, X, "matern32", ells, oss)
    Kf = ok.full_kernel_cn_per_class(Ks)
    # entry by entry from the definition
    for (n, c, m, c2) in [(0, 0, 0, 0), (3, 1, 7, 1), (5, 2, 5, 2), (4, 0, 9, 2), (2, 1, 2, 0)]:
        want = ok.kernel_matrix(X[n:n + 1], X[m:m + 1], "matern32", ells[c], oss[c])[0, 0] \
            if c == c2 else 0.0
        assert abs(Kf[n * 3 + c, m * 3 + c2] - want) < 1e-15
    assert np.allclose(Kf, Kf.T) and np.linalg.eigvalsh(Kf).min() > -1e-10
    assert np.allclose(np.diag(Kf), np.tile(oss, 30))
    v = rng.standard_normal((90, 4))
    np.testing.assert_allclose(ok.apply_kernel_per_class(Ks, v), Kf @ v, rtol=1e-13, atol=1e-13)
    Ks1 = ok.kernel_matrices_per_class(X, X, "rbf", [0.9] * 3, [1.2] * 3)
    np.testing.assert_allclose(ok.full_kernel_cn_per_class(Ks1),
                               ok.full_kernel_cn(ok.kernel_matrix(X, X, "rbf", 0.9, 1.2), 3),
                               rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("kind", ["rbf", "matern32", "matern52"])
def test_gram_form_matches_explicit_differences(kind):
    """The norm-expansion form of the kernel matrix (used for many features)
    against the explicit-difference definition, within the rounding of the
    expansion: |dr^2| <= 2 D eps (|x1|^2 + |x2|^2) / l^2 and |dk| <= L |dr^2|
    with L = max |dk/d(r^2)| / os (1/2 RBF, 3/2 Matern-3/2, 5/6 Matern-5/2)."""
    rng = np.random.default_rng(41)
    D = 784
    X1 = rng.uniform(0.0, 1.0, size=(150, D)) * (rng.uniform(size=(150, D)) < 0.2)
    X2 = rng.uniform(0.0, 1.0, size=(90, D)) * (rng.uniform(size=(90, D)) < 0.2)
    X2[:5] = X1[:5]                               # coincident points (r = 0)
    ell, os_ = 7.5, 1.7
    ref = ok.kernel_matrix(X1, X2, kind, ell, os_)
    got = ok.kernel_matrix_gram(X1, X2, kind, ell, os_, block=64)
    lip = {"rbf": 0.5, "matern32": 1.5, "matern52": 5.0 / 6.0}[kind]
    eps = np.finfo(np.float64).eps
    nn = (X1 * X1).sum(1)[:, None] + (X2 * X2).sum(1)[None, :]
    bound = os_ * lip * 2.0 * D * eps * nn / ell ** 2
    assert np.all(np.abs(got - ref) <= bound + 4 * eps * os_)
    # a wrong factor in the expansion is far outside that bound
    assert np.abs(got - ref).max() < 1e-10
