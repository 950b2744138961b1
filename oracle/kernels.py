"""Kernel functions, FP64, plain definitions.

The paper names the kernels (RBF for the toy and Poisson experiments,
Matern-3/2 for the Gaussian-mixture and MNIST experiments; appendix on
experimental details) with a lengthscale and an outputscale.  We read the
outputscale as a multiplicative variance (GPyTorch's ScaleKernel) and use the
textbook forms (Rasmussen & Williams 2006, Sec. 4.2) with r = ||x - x'|| / l:

    RBF         os * exp(-r^2 / 2)
    Matern-1/2  os * exp(-r)
    Matern-3/2  os * (1 + sqrt(3) r) exp(-sqrt(3) r)
    Matern-5/2  os * (1 + sqrt(5) r + 5 r^2 / 3) exp(-sqrt(5) r)

Distances are formed from explicit coordinate differences (no norm
expansion), so the diagonal of K(X, X) is exactly os.

Pins (tests/test_oracle_kernels.py): the Matern forms against the general
Bessel-function definition (scipy.special.kv); RBF against the Gaussian
density (scipy.stats.norm); brute-force double loop; symmetry, PSD, diagonal.
"""
from __future__ import annotations

import math

import numpy as np

KINDS = ("rbf", "matern12", "matern32", "matern52")


def scaled_sqdist(X1: np.ndarray, X2: np.ndarray, lengthscale: float) -> np.ndarray:
    """r^2 = ||x1 - x2||^2 / l^2 from explicit differences, shape (N1, N2)."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    r2 = np.zeros((X1.shape[0], X2.shape[0]))
    for d in range(X1.shape[1]):
        diff = X1[:, d, None] - X2[None, :, d]
        r2 += diff * diff
    return r2 / (lengthscale * lengthscale)


def kernel_of_r2(r2: np.ndarray, kind: str, outputscale: float) -> np.ndarray:
    """Stationary kernel value as a function of the scaled squared distance."""
    r2 = np.asarray(r2, dtype=np.float64)
    if kind == "rbf":
        return outputscale * np.exp(-0.5 * r2)
    r = np.sqrt(r2)
    if kind == "matern12":
        return outputscale * np.exp(-r)
    if kind == "matern32":
        a = math.sqrt(3.0) * r
        return outputscale * (1.0 + a) * np.exp(-a)
    if kind == "matern52":
        a = math.sqrt(5.0) * r
        return outputscale * (1.0 + a + a * a / 3.0) * np.exp(-a)
    raise ValueError(f"unknown kernel {kind!r}")


def kernel_matrix(X1, X2, kind: str, lengthscale: float, outputscale: float,
                  block: int = 2048) -> np.ndarray:
    """K_X[n, m] = k(x1_n, x2_m), shape (N1, N2), FP64."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    out = np.empty((X1.shape[0], X2.shape[0]))
    for i0 in range(0, X1.shape[0], block):
        out[i0:i0 + block] = kernel_of_r2(
            scaled_sqdist(X1[i0:i0 + block], X2, lengthscale), kind, outputscale)
    return out


def kernel_matrix_gram(X1, X2, kind: str, lengthscale: float, outputscale: float,
                       out: np.ndarray = None, block: int = 4096) -> np.ndarray:
    """K_X[n, m] = k(x1_n, x2_m) with the squared distance expanded as
    |x1|^2 + |x2|^2 - 2 x1.x2 (FP64, one matrix product per row block, clamped
    at 0).  For many features (hundreds), where the explicit differences of
    ``kernel_matrix`` cost one pass over the block per feature.  The expansion
    changes r^2 by at most about 2 D eps_64 (|x1|^2 + |x2|^2) / l^2 (pinned
    against ``kernel_matrix``).  ``out`` may be a preallocated (N1, N2) array."""
    X1 = np.asarray(X1, dtype=np.float64)
    X2 = np.asarray(X2, dtype=np.float64)
    if out is None:
        out = np.empty((X1.shape[0], X2.shape[0]))
    n2 = (X2 * X2).sum(axis=1)
    inv_l2 = 1.0 / (lengthscale * lengthscale)
    for i0 in range(0, X1.shape[0], block):
        A = X1[i0:i0 + block]
        r2 = A @ X2.T
        r2 *= -2.0
        r2 += (A * A).sum(axis=1)[:, None]
        r2 += n2[None, :]
        np.maximum(r2, 0.0, out=r2)
        r2 *= inv_l2
        out[i0:i0 + block] = kernel_of_r2(r2, kind, outputscale)
    return out


def kernel_matvec(X1, X2, V, kind: str, lengthscale: float, outputscale: float,
                  block: int = 1024) -> np.ndarray:
    """Out = K_X(X1, X2) @ V for V of shape (N2, W), blockwise over rows of X1
    so that K is never held whole (the paper's lazily evaluated product with K,
    appendix on matrix-vector products)."""
    X1 = np.asarray(X1, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    out = np.empty((X1.shape[0],) + V.shape[1:])
    for i0 in range(0, X1.shape[0], block):
        Kb = kernel_matrix(X1[i0:i0 + block], X2, kind, lengthscale, outputscale)
        out[i0:i0 + block] = Kb @ V
    return out


def full_kernel_cn(KX: np.ndarray, C: int) -> np.ndarray:
    """The NC x NC prior covariance in CN-ordering (index n*C + c) when the C
    latent functions are independent GPs sharing one kernel: K = K_X (x) I_C.
    (Appendix on orderings: K is block diagonal in NC-ordering; re-indexed to
    CN-ordering it is the Kronecker product with the identity on the right.)"""
    return np.kron(KX, np.eye(C))


def apply_full_kernel_cn(KX: np.ndarray, v: np.ndarray, C: int) -> np.ndarray:
    """(K_X (x) I_C) v for CN-ordered v of length N*C (or shape (N*C, b))."""
    N = KX.shape[0]
    if v.ndim == 1:
        return (KX @ v.reshape(N, C)).reshape(-1)
    b = v.shape[1]
    return np.einsum("nm,mcb->ncb", KX, v.reshape(N, C, b)).reshape(N * C, b)


# --- one kernel per latent function ------------------------------------------

def kernel_matrices_per_class(X1, X2, kind: str, lengthscales, outputscales):
    """K_c(X1, X2) for c < C: the same kernel family with class-specific
    lengthscale and outputscale (independent GPs with their own
    hyperparameters)."""
    return [kernel_matrix(X1, X2, kind, l, o) for l, o in zip(lengthscales, outputscales)]


def full_kernel_cn_per_class(Ks) -> np.ndarray:
    """The NC x NC prior covariance in CN-ordering for C independent GPs with
    kernels K_c: entry (n*C + c, m*C + c') = delta_{c c'} K_c[n, m], i.e.
    sum_c K_c (x) e_c e_c^T."""
    C = len(Ks)
    N, M = Ks[0].shape
    out = np.zeros((N * C, M * C))
    for c, K in enumerate(Ks):
        E = np.zeros((C, C))
        E[c, c] = 1.0
        out += np.kron(K, E)
    return out


def apply_kernel_per_class(Ks, v: np.ndarray) -> np.ndarray:
    """(sum_c K_c (x) e_c e_c^T) v for CN-ordered v of length M*C (or (M*C, b))."""
    C = len(Ks)
    N, M = Ks[0].shape
    V = v.reshape(M, C, -1)
    out = np.stack([Ks[c] @ V[:, c, :] for c in range(C)], axis=1)   # (N, C, b)
    return out.reshape(N * C) if v.ndim == 1 else out.reshape(N * C, -1)
