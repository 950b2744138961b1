"""Pins for oracle.likelihood: finite differences, numpy pinv, Moore-Penrose."""
import numpy as np
import pytest

from oracle import likelihood as lk


def _problem(seed=0, N=7, C=4, scale=2.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, C)) * scale, rng.integers(0, C, size=N)


def test_softmax_normalised_and_stable():
    F = np.array([[1000.0, 999.0, -1000.0], [0.0, 0.0, 0.0]])
    P = lk.softmax(F)
    np.testing.assert_allclose(P.sum(1), 1.0, rtol=1e-13)
    np.testing.assert_allclose(P[1], 1.0 / 3.0, rtol=1e-15)
    np.testing.assert_allclose(P[0, 0] / P[0, 1], np.e, rtol=1e-12)


def test_gradient_matches_finite_differences():
    F, y = _problem()
    g = lk.softmax_grad(F, y)
    h = 1e-6
    fd = np.zeros_like(F)
    for n in range(F.shape[0]):
        for c in range(F.shape[1]):
            Fp, Fm = F.copy(), F.copy()
            Fp[n, c] += h
            Fm[n, c] -= h
            fd[n, c] = (lk.softmax_loglik(Fp, y) - lk.softmax_loglik(Fm, y)) / (2 * h)
    np.testing.assert_allclose(g, fd, atol=1e-8)


def test_hessian_blocks_match_finite_differences():
    F, y = _problem(1)
    W = lk.softmax_hessian_blocks(F)
    h = 1e-5
    N, C = F.shape
    for n in range(N):
        for c in range(C):
            Fp, Fm = F.copy(), F.copy()
            Fp[n, c] += h
            Fm[n, c] -= h
            col = (lk.softmax_grad(Fp, y) - lk.softmax_grad(Fm, y)) / (2 * h)
            # -d grad / d f = W; only the block of point n is non-zero
            np.testing.assert_allclose(-col[n], W[n, :, c], atol=1e-9)
            other = np.delete(col, n, axis=0)
            assert np.abs(other).max() == 0.0


def test_hessian_blocks_psd_rows_sum_to_zero():
    F, _ = _problem(2, N=20, C=5)
    W = lk.softmax_hessian_blocks(F)
    np.testing.assert_allclose(W.sum(axis=2), 0.0, atol=1e-15)
    for n in range(20):
        assert np.allclose(W[n], W[n].T)
        lam = np.linalg.eigvalsh(W[n])
        assert lam.min() >= -1e-15
        assert np.sum(lam > 1e-12) == 4          # rank C - 1


@pytest.mark.parametrize("C", [2, 3, 5, 10])
def test_pinv_lemma_matches_numpy_pinv_and_penrose(C):
    F, _ = _problem(3, N=12, C=C, scale=1.5)
    W = lk.softmax_hessian_blocks(F)
    Wp = lk.softmax_hessian_pinv_blocks(F)
    P = np.eye(C) - np.ones((C, C)) / C
    for n in range(F.shape[0]):
        A, G = W[n], Wp[n]
        ref = np.linalg.pinv(A, rcond=1e-13)
        np.testing.assert_allclose(G, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
        np.testing.assert_allclose(A @ G @ A, A, atol=1e-12)
        np.testing.assert_allclose(G @ A @ G, G, rtol=1e-11, atol=1e-11 * np.abs(G).max())
        np.testing.assert_allclose(A @ G, (A @ G).T, atol=1e-12)
        np.testing.assert_allclose(G @ A, (G @ A).T, atol=1e-12)
        np.testing.assert_allclose(A @ G, P, atol=1e-12)
        np.testing.assert_allclose(G @ np.ones(C), 0.0, atol=1e-12 * np.abs(G).max())


def test_apply_blocks_equals_dense():
    F, _ = _problem(4, N=5, C=3)
    Wp = lk.softmax_hessian_pinv_blocks(F)
    D = lk.dense_block_diag(Wp)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(15)
    M = rng.standard_normal((15, 4))
    np.testing.assert_allclose(lk.apply_blocks(Wp, v), D @ v, rtol=1e-13)
    np.testing.assert_allclose(lk.apply_blocks(Wp, M), D @ M, rtol=1e-13)


def test_poisson_derivatives_match_finite_differences():
    rng = np.random.default_rng(6)
    f = rng.standard_normal(9)
    y = rng.poisson(2.0, size=9)
    h = 1e-6
    fd = np.array([(lk.poisson_loglik(f + h * e, y) - lk.poisson_loglik(f - h * e, y)) / (2 * h)
                   for e in np.eye(9)])
    np.testing.assert_allclose(lk.poisson_grad(f, y), fd, atol=1e-7)
    hd = np.array([(lk.poisson_grad(f + h * e, y) - lk.poisson_grad(f - h * e, y)) / (2 * h)
                   for e in np.eye(9)])
    np.testing.assert_allclose(np.diag(-hd), 1.0 / lk.poisson_winv_diag(f), rtol=1e-7)
