"""Predictions, FP64.

IterGP posterior after solver iteration j of Newton step i (paper eqs. for
m_{i,j} and k_{i,j}, Section 3.1), with all classes sharing one kernel so that
K(x, X) = K_X(x, X) (x) I_C in CN-ordering:

    mean[s, c] = m + sum_n k(xs, x_n) v[n*C + c]
    var[s, c]  = k(xs, xs) - sum_b ( sum_n k(xs, x_n) Q[n*C + c, b] )^2

The variance line is the diagonal of k(xs, xs) - K(xs, X) Q Q^T K(X, xs) with
C_j = Q Q^T.  The exact Laplace predictive (eq. for k_{i,*}) replaces Q Q^T by
Khat^{-1}.  Predictive class probabilities use the probit approximation
softmax(mean / sqrt(1 + pi/8 var)) (appendix on the large-scale experiment).

Pins (tests/test_oracle_predict.py): at full budget the IterGP variance equals
the exact variance; the variance is non-increasing in j (Proposition "The
Uncertainty Decreases in the Inner Loop"); probit with var = 0 is the softmax
of the mean; in the binary case the scale applied to the mean equals the
exact Gaussian smoothing of the cdf Phi(lam x) whose slope at 0 matches the
sigmoid's (checked by adaptive quadrature), and the result is within twice
the sigmoid-to-cdf substitution error of the logistic-normal integral.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .kernels import kernel_matrix


def predictive_mean(Xs, X, v, C, kind, ell, os_):
    Ks = kernel_matrix(Xs, X, kind, ell, os_)
    return Ks @ v.reshape(X.shape[0], C)


def predictive_var_root(Xs, X, Q, C, kind, ell, os_):
    """Marginal variances with C_j = Q Q^T, shape (Ns, C)."""
    Ks = kernel_matrix(Xs, X, kind, ell, os_)
    N = X.shape[0]
    b = Q.shape[1]
    A = np.einsum("sn,ncb->scb", Ks, Q.reshape(N, C, b))
    return os_ - (A * A).sum(axis=2)


def predictive_var_exact(Xs, X, Khat, C, kind, ell, os_):
    """Marginal variances of the Laplace predictive with Khat^{-1}, (Ns, C)."""
    Ks = kernel_matrix(Xs, X, kind, ell, os_)
    Kf = np.kron(Ks, np.eye(C))                     # (Ns*C, N*C)
    cf = sla.cho_factor(Khat, lower=True)
    sol = sla.cho_solve(cf, Kf.T)
    red = np.einsum("ij,ji->i", Kf, sol)
    return (os_ - red).reshape(Xs.shape[0], C)


def predictive_mean_per_class(Xs, X, v, kind, lengthscales, outputscales):
    """Mean with one kernel per latent function: mean[s, c] = sum_n k_c(xs, x_n) v[n*C + c]."""
    C = len(lengthscales)
    V = v.reshape(X.shape[0], C)
    return np.stack([kernel_matrix(Xs, X, kind, l, o) @ V[:, c]
                     for c, (l, o) in enumerate(zip(lengthscales, outputscales))], axis=1)


def predictive_var_root_per_class(Xs, X, Q, kind, lengthscales, outputscales):
    """Marginal variances with C_j = Q Q^T and one kernel per latent function:
    var[s, c] = k_c(xs, xs) - sum_b (sum_n k_c(xs, x_n) Q[n*C + c, b])^2."""
    C = len(lengthscales)
    N, b = X.shape[0], Q.shape[1]
    Qr = Q.reshape(N, C, b)
    out = []
    for c, (l, o) in enumerate(zip(lengthscales, outputscales)):
        A = kernel_matrix(Xs, X, kind, l, o) @ Qr[:, c, :]
        out.append(o - (A * A).sum(axis=1))
    return np.stack(out, axis=1)


def probit_probs(mean: np.ndarray, var: np.ndarray) -> np.ndarray:
    z = mean / np.sqrt(1.0 + (math.pi / 8.0) * var)
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def accuracy(probs: np.ndarray, y: np.ndarray) -> float:
    return float((probs.argmax(axis=1) == np.asarray(y)).mean())


def nll(probs: np.ndarray, y: np.ndarray) -> float:
    """Mean negative log predictive probability of the true class."""
    return float(-np.log(probs[np.arange(len(y)), np.asarray(y)]).mean())
