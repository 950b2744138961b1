"""Likelihood pieces, FP64, plain definitions.

Softmax (categorical) likelihood for C classes, CN-ordered latent vector f of
length N*C viewed as an (N, C) array F (paper Sec. 2.1 and the appendix on
orderings):

    pi_n      = softmax(F_n)                      (log-sum-exp form)
    grad      = onehot(y) - pi                    (gradient of log p(y|f))
    W_n       = diag(pi_n) - pi_n pi_n^T          (negative Hessian block)
    W_n^+     = P diag(1 / pi_n) P,  P = I - 11^T / C

The last line is the paper's explicit pseudo-inverse (appendix lemma on the
pseudo-inverse for multi-class classification); W is block diagonal with N
blocks of size C x C in CN-ordering.  The lemma's final formula is correct,
but two intermediate identities printed in its proof are not (one drops a
diag, one claims diag(1/pi) A_n = I, which in fact equals I - 1 pi^T); this
file follows only the final formula.

Poisson (C = 1): grad = y - exp(f), W^{-1} = diag(exp(-f))  (appendix on the
Poisson log likelihood).  Gaussian with noise variances lam: W^{-1} = diag(lam),
pseudo-targets equal y (Theorem "Generalization of IterGP").

Pins (tests/test_oracle_likelihood.py): gradient and Hessian against central
finite differences of log p(y|f); W^+ against numpy.linalg.pinv and the four
Moore-Penrose conditions; W_n 1 = 0; W_n PSD.
"""
from __future__ import annotations

import numpy as np


def log_softmax(F: np.ndarray) -> np.ndarray:
    F = np.asarray(F, dtype=np.float64)
    mx = F.max(axis=1, keepdims=True)
    lse = mx + np.log(np.exp(F - mx).sum(axis=1, keepdims=True))
    return F - lse


def softmax(F: np.ndarray) -> np.ndarray:
    return np.exp(log_softmax(F))


def onehot(y: np.ndarray, C: int) -> np.ndarray:
    Y = np.zeros((len(y), C))
    Y[np.arange(len(y)), np.asarray(y)] = 1.0
    return Y


def softmax_loglik(F: np.ndarray, y: np.ndarray) -> float:
    """log p(y | f) = sum_n log pi_n[y_n]."""
    ls = log_softmax(F)
    return float(ls[np.arange(len(y)), np.asarray(y)].sum())


def softmax_grad(F: np.ndarray, y: np.ndarray) -> np.ndarray:
    """grad log p(y|f) as an (N, C) array: onehot(y) - pi."""
    return onehot(y, F.shape[1]) - softmax(F)


def softmax_hessian_blocks(F: np.ndarray) -> np.ndarray:
    """W_n = diag(pi_n) - pi_n pi_n^T, shape (N, C, C)."""
    P = softmax(F)
    return np.einsum("nc,cd->ncd", P, np.eye(F.shape[1])) - np.einsum("nc,nd->ncd", P, P)


def softmax_hessian_pinv_blocks(F: np.ndarray) -> np.ndarray:
    """W_n^+ = (I - 11^T/C) diag(1/pi_n) (I - 11^T/C), shape (N, C, C)."""
    C = F.shape[1]
    P = softmax(F)
    Pc = np.eye(C) - np.ones((C, C)) / C
    D = np.einsum("nc,cd->ncd", 1.0 / P, np.eye(C))
    return np.einsum("ij,njk,kl->nil", Pc, D, Pc)


def apply_blocks(B: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Block-diagonal product for CN-ordered v (length N*C or (N*C, b))."""
    N, C, _ = B.shape
    if v.ndim == 1:
        return np.einsum("nij,nj->ni", B, v.reshape(N, C)).reshape(-1)
    b = v.shape[1]
    return np.einsum("nij,njb->nib", B, v.reshape(N, C, b)).reshape(N * C, b)


def dense_block_diag(B: np.ndarray) -> np.ndarray:
    """The NC x NC matrix with the N blocks on its diagonal (small N only)."""
    N, C, _ = B.shape
    out = np.zeros((N * C, N * C))
    for n in range(N):
        out[n * C:(n + 1) * C, n * C:(n + 1) * C] = B[n]
    return out


# --- Poisson regression (C = 1) -------------------------------------------------

def poisson_loglik(f: np.ndarray, y: np.ndarray) -> float:
    """sum_n y_n f_n - exp(f_n) - log(y_n!)"""
    from scipy.special import gammaln
    f = np.asarray(f, dtype=np.float64)
    return float((y * f - np.exp(f) - gammaln(np.asarray(y) + 1.0)).sum())


def poisson_grad(f: np.ndarray, y: np.ndarray) -> np.ndarray:
    return np.asarray(y, dtype=np.float64) - np.exp(f)


def poisson_winv_diag(f: np.ndarray) -> np.ndarray:
    """Diagonal of W(f)^{-1} = diag(exp(-f))."""
    return np.exp(-np.asarray(f, dtype=np.float64))
