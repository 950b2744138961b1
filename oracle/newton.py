"""O-exact: Newton steps of the multi-class Laplace problem, FP64, dense.

The paper rewrites a Newton step on the log posterior Psi (its eq. for the
Newton step) as the solve of a GP-regression system (Proposition
"Reformulation of the Newton Step" and Section 3.1):

    yhat - m = (f_i - m) + W(f_i)^+ grad log p(y | f_i)     (pseudo-targets)
    (K + W(f_i)^+) v = yhat - m                            (Khat v = yhat - m)
    f_{i+1} = K v + m

with the pseudo-inverse substituted where W is singular (Section 3.1
footnote).  This file writes that definition out with a dense Cholesky
(scipy.linalg.cho_factor) of Khat, for small N only.  m = 0 throughout (zero
prior mean in every experiment of the paper).

``textbook_newton_step`` is the plain Newton update
f_{i+1} = f_i - (grad^2 Psi)^{-1} grad Psi with grad^2 Psi = -W - K^{-1} (the
paper's eq. for the Newton step), formed with explicit inverses -- an
independent route used to pin ``exact_step`` when all classes share one
kernel.

Pins (tests/test_oracle_newton.py): equality with the textbook Newton step;
the fixed point f* = K grad log p(y | f*) of the mode; monotone increase of
Psi; the mode found by a generic optimiser on tiny N; for a Gaussian
likelihood, one step reaches the exact posterior mean (Theorem
"Generalization of IterGP").
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import likelihood as lik


def pseudo_target_offset(F: np.ndarray, y: np.ndarray) -> np.ndarray:
    """yhat - m = g + W^+ (onehot(y) - pi) with g = f - m = f (m = 0);
    CN-ordered vector of length N*C."""
    Wp = lik.softmax_hessian_pinv_blocks(F)
    b = lik.softmax_grad(F, y).reshape(-1)
    return F.reshape(-1) + lik.apply_blocks(Wp, b)


def khat_dense(K_full: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Khat = K + W(f)^+ as a dense NC x NC matrix."""
    return K_full + lik.dense_block_diag(lik.softmax_hessian_pinv_blocks(F))


def exact_step(K_full: np.ndarray, F: np.ndarray, y: np.ndarray):
    """One exact Newton step.  Returns (F_next (N, C), v (NC,), rhs (NC,))."""
    N, C = F.shape
    rhs = pseudo_target_offset(F, y)
    cf = sla.cho_factor(khat_dense(K_full, F), lower=True)
    v = sla.cho_solve(cf, rhs)
    return (K_full @ v).reshape(N, C), v, rhs


def exact_newton(K_full: np.ndarray, y: np.ndarray, C: int, steps: int, F0=None):
    """Run ``steps`` exact Newton steps from f_0 = m = 0.  Returns the list of
    iterates [F_0, ..., F_steps] and of representer weights [v_0 .. v_{steps-1}]."""
    N = K_full.shape[0] // C
    F = np.zeros((N, C)) if F0 is None else np.array(F0, dtype=np.float64)
    Fs, vs = [F], []
    for _ in range(steps):
        F, v, _ = exact_step(K_full, F, y)
        Fs.append(F)
        vs.append(v)
    return Fs, vs


def textbook_newton_step(K_full: np.ndarray, F: np.ndarray, y: np.ndarray) -> np.ndarray:
    """f - (grad^2 Psi)^{-1} grad Psi with the true (singular-W) Hessian."""
    N, C = F.shape
    f = F.reshape(-1)
    Kinv = np.linalg.inv(K_full)
    W = lik.dense_block_diag(lik.softmax_hessian_blocks(F))
    grad = lik.softmax_grad(F, y).reshape(-1) - Kinv @ f
    hess = -W - Kinv
    return (f - np.linalg.solve(hess, grad)).reshape(N, C)


def log_posterior(K_full: np.ndarray, F: np.ndarray, y: np.ndarray) -> float:
    """Psi(f) = log p(y|f) - 1/2 (f - m)^T K^{-1} (f - m) (up to a constant)."""
    f = F.reshape(-1)
    return lik.softmax_loglik(F, y) - 0.5 * float(f @ np.linalg.solve(K_full, f))


def psi_from_v(F: np.ndarray, y: np.ndarray, v: np.ndarray) -> float:
    """Psi at f = K v + m via g^T K^{-1} g = g^T v (because g = K v)."""
    return lik.softmax_loglik(F, y) - 0.5 * float(F.reshape(-1) @ v)


# --- general diagonal-noise problems (Poisson, Gaussian) ----------------------

def exact_step_diag(K: np.ndarray, f: np.ndarray, grad: np.ndarray,
                    winv_diag: np.ndarray):
    """Newton step for a likelihood with diagonal W^{-1} (C = 1):
    yhat - m = f + W^{-1} grad; (K + W^{-1}) v = yhat - m; f_next = K v."""
    rhs = f + winv_diag * grad
    cf = sla.cho_factor(K + np.diag(winv_diag), lower=True)
    v = sla.cho_solve(cf, rhs)
    return K @ v, v, rhs
