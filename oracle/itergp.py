"""O-method: IterNCGP (Algorithm 1), IterGP (Algorithm 2) and the virtual
solver run with compression (Algorithm 3), FP64, matrix-free.

Written from the paper's statement of the method in its notation: actions
s_j, products t_j = K s_j, buffers S and T, the approximate precision matrix
C_j = S_j (S_j^T Khat S_j)^{-1} S_j^T (eq. C_j) with root Q, representer
weights v_j = C_j (yhat - m), normaliser eta_j and observation alpha_j.  The
inner solve is written from the definition of C_j (a Cholesky factor of the
Gram matrix of the actions, grown by one row per action), not from the
recurrence for the search direction that Algorithm 2 uses to update it; the
two agree in exact arithmetic, and the library implements the recurrence.

Readings of points the paper leaves open:

* The inner stopping test uses ||r_{j-1}|| right after it is formed, before
  an action is chosen; the iteration cap is tested before the residual is
  formed, so no product with K is spent on a residual that cannot be used.
  Tolerances: ||r|| < max(tol_abs, tol_rel ||yhat - m||), both 1e-5 by
  default (appendix on stopping criteria).
* CG actions are stored normalised, s_j = r_{j-1} / ||r_{j-1}||.  All outputs
  are invariant to the scale of an action (C_j depends only on span S); the
  invariance is pinned by a test.
* eta_j <= 0 ends the solve (appendix on stopping criteria); that action and
  its product are not kept in S and T (Algorithm 2 appends them before eta_j
  is known), so the recycled M of the next Newton step stays nonsingular.
* Algorithm 3 takes M = S^T (T + W^+ S), symmetrised as (M + M^T)/2, and its
  eigenpairs sorted by decreasing eigenvalue.  Eigenpairs with
  lambda <= lambda_max * B * eps_64 are dropped before truncation to R
  (the paper takes Lambda^{-1/2} without guarding against tiny eigenvalues).
* The unit-vector policy restarts at e_1 in every Newton step and runs
  without recycling (the paper's Cholesky runs are without recycling).

Likelihoods with a diagonal negative Hessian (Poisson with log link,
Gaussian) run the same loop with W^{-1} diagonal (iterncgp_diag); any
likelihood that factorises over the points, given as its gradient and C x C
negative-Hessian blocks, with W^{-1} block diagonal (iterncgp_block).

Pins (tests/test_oracle_itergp.py): full-budget IterGP equals the dense
Cholesky solve; C_j = S (S^T Khat S)^{-1} S^T equals Q Q^T; the unit policy
equals exact GP regression on the leading coordinates; the residual policy
equals textbook conjugate gradients (scipy.sparse.linalg.cg); S^T r_j = 0;
after the virtual solver run S^T r_0 = 0 and the Khat-projected error is zero;
R = 0 gives C_0 = 0; the marginal variance is non-increasing in j; the
trace identity Tr K_{i,0} = Tr K - Tr M for eigenvector actions with
W^{-1} = 0.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

from . import likelihood as lik
from .newton import pseudo_target_offset

Apply = Callable[[np.ndarray], np.ndarray]
EPS64 = np.finfo(np.float64).eps


@dataclasses.dataclass
class VSRInfo:
    eigvals: np.ndarray          # kept eigenvalues (descending)
    n_dropped_floor: int = 0     # eigenpairs removed by the tiny-eigenvalue floor
    n_dropped_rank: int = 0      # eigenpairs removed by compression to R


@dataclasses.dataclass
class SolveInfo:
    iters: int = 0                       # new actions taken (j at exit)
    res_norms: List[float] = dataclasses.field(default_factory=list)
    etas: List[float] = dataclasses.field(default_factory=list)
    alphas: List[float] = dataclasses.field(default_factory=list)
    actions: List[np.ndarray] = dataclasses.field(default_factory=list)
    breakdown: bool = False
    converged: bool = False
    rhs_norm: float = 0.0
    vsr: Optional[VSRInfo] = None


def virtual_solver_run(S: np.ndarray, T: np.ndarray, apply_Winv: Apply,
                       rank_limit: Optional[int] = None):
    """Algorithm 3.  Returns (Q0, S, T, info) with C_0 = Q0 Q0^T.

    M = S^T (T + W^{-1} S) = S^T Khat S; M = U Lambda U^T with eigenvalues in
    decreasing order; keep the R largest (compression); S <- S U, T <- T U;
    Q0 = S Lambda^{-1/2}.
    """
    B = S.shape[1]
    if B == 0:
        return S.copy(), S.copy(), T.copy(), VSRInfo(np.zeros(0))
    M = S.T @ (T + apply_Winv(S))
    M = 0.5 * (M + M.T)
    lam, U = np.linalg.eigh(M)
    order = np.argsort(lam)[::-1]
    lam, U = lam[order], U[:, order]
    keep = lam > lam[0] * B * EPS64 if lam[0] > 0 else np.zeros(B, dtype=bool)
    n_floor = int(B - keep.sum())
    lam, U = lam[keep], U[:, keep]
    n_rank = 0
    if rank_limit is not None and rank_limit >= 0 and lam.size > rank_limit:
        n_rank = int(lam.size - rank_limit)
        lam, U = lam[:rank_limit], U[:, :rank_limit]
    S = S @ U
    T = T @ U
    Q0 = S / np.sqrt(lam)[None, :]
    return Q0, S, T, VSRInfo(lam, n_floor, n_rank)


def _choose_action(policy: str, r: np.ndarray, rn: float, j: int,
                   user_actions: Optional[np.ndarray], normalize: bool) -> np.ndarray:
    """The policy's j-th action (1-based) given the current residual r."""
    if policy == "cg":                     # residual actions: CG in exact arithmetic
        return r / rn if normalize else r.copy()
    if policy == "unit":                   # unit vectors: partial Cholesky / subset of data
        e = np.zeros(r.shape[0])
        e[j - 1] = 1.0
        return e
    if policy == "user":
        return np.array(user_actions[:, j - 1], dtype=np.float64)
    raise ValueError(policy)


def itergp(apply_K: Apply, apply_Winv: Apply, rhs: np.ndarray,
           S: np.ndarray, T: np.ndarray, policy: str = "cg", j_max: int = 100,
           tol_abs: float = 1e-5, tol_rel: float = 1e-5,
           rank_limit: Optional[int] = None, recycle: bool = True,
           user_actions: Optional[np.ndarray] = None,
           normalize_actions: bool = True):
    """IterGP (Algorithm 2) for the system Khat v = rhs (rhs = yhat - m), with
    Khat = K + W^{-1}.

    The method's state after j actions is the approximate precision matrix of
    eq. C_j, C_j = S_j (S_j^T Khat S_j)^{-1} S_j^T, and the representer
    weights v_j = C_j rhs.  This function writes that definition out: the
    Gram matrix M_j = S_j^T Khat S_j = S_j^T (T_j + W^{-1} S_j) (T_j = K S_j,
    kept beside S_j) is grown by one row and column per action, factored
    M_j = L_j L_j^T, and v_j = S_j M_j^{-1} S_j^T rhs.  The new action is chosen
    from the residual r_{j-1} = rhs - Khat v_{j-1}.  The last pivot of L_j,
    eta_j = (M_j)_{jj} - |L_{j-1}^{-1} (M_j)_{1:j-1, j}|^2, is the Schur
    complement of the new action against the previous ones (the normaliser of
    the search direction in Algorithm 2); eta_j <= 0 means the action adds no
    direction in the Khat geometry, which ends the solve.  The returned root Q
    of C_j is S_j L_j^{-T}.  With recycling, S_0 and T_0 come from the virtual
    solver run (Algorithm 3) and C_0 = S_0 (S_0^T Khat S_0)^{-1} S_0^T is the
    initial precision matrix of the step.

    Returns (v, Q, S, T, info).  ``policy`` is "cg" (s_j = r_{j-1}), "unit"
    (s_j = e_j) or "user" (s_j = user_actions[:, j-1]; the solve ends when the
    supplied actions are used up).
    """
    n = rhs.shape[0]
    if recycle:
        _, S, T, vinfo = virtual_solver_run(S, T, apply_Winv, rank_limit)
    else:
        S, T, vinfo = np.zeros((n, 0)), np.zeros((n, 0)), None
    info = SolveInfo(vsr=vinfo)
    cols_S, cols_T = [S[:, k] for k in range(S.shape[1])], [T[:, k] for k in range(T.shape[1])]
    b0 = len(cols_S)
    M = S.T @ (T + apply_Winv(S)) if b0 else np.zeros((0, 0))
    M = 0.5 * (M + M.T)
    L = np.linalg.cholesky(M) if b0 else np.zeros((0, 0))
    proj = S.T @ rhs                                     # S_j^T rhs

    def weights():
        """v_j = S_j M_j^{-1} S_j^T rhs through the factor L_j."""
        if not cols_S:
            return np.zeros(n)
        w = sla.solve_triangular(L, proj, lower=True)
        w = sla.solve_triangular(L.T, w, lower=False)
        return np.stack(cols_S, axis=1) @ w

    v = weights()
    rhs_norm = float(np.linalg.norm(rhs))
    info.rhs_norm = rhs_norm
    thresh = max(tol_abs, tol_rel * rhs_norm)
    j = 0
    while j < j_max:
        r = rhs - apply_K(v) - apply_Winv(v)
        rn = float(np.linalg.norm(r))
        info.res_norms.append(rn)
        if rn < thresh:
            info.converged = True
            break
        if policy == "user" and j >= user_actions.shape[1]:
            break
        s = _choose_action(policy, r, rn, j + 1, user_actions, normalize_actions)
        t = apply_K(s)
        ks = t + apply_Winv(s)                           # Khat s
        # new row/column of the Gram matrix and the Schur complement of s
        m_new = np.array([c @ ks for c in cols_S])
        mu = float(s @ ks)
        l_new = (sla.solve_triangular(L, m_new, lower=True) if cols_S else np.zeros(0))
        eta = mu - float(l_new @ l_new)
        if eta <= 0.0:
            info.breakdown = True                        # s is dropped again
            break
        j += 1
        info.alphas.append(float(s @ r))
        info.etas.append(eta)
        info.actions.append(s)
        cols_S.append(s)
        cols_T.append(t)
        k = L.shape[0]
        L2 = np.zeros((k + 1, k + 1))
        L2[:k, :k] = L
        L2[k, :k] = l_new
        L2[k, k] = np.sqrt(eta)
        L = L2
        proj = np.append(proj, s @ rhs)
        v = weights()
    info.iters = j
    S = np.stack(cols_S, axis=1) if cols_S else np.zeros((n, 0))
    T = np.stack(cols_T, axis=1) if cols_T else np.zeros((n, 0))
    Q = sla.solve_triangular(L, S.T, lower=True).T if cols_S else np.zeros((n, 0))
    return v, Q, S, T, info


@dataclasses.dataclass
class NewtonRecord:
    F: np.ndarray          # iterate after the step, (N, C)
    v: np.ndarray          # representer weights of the step
    Q: np.ndarray          # root of C_j at the end of the step
    rhs: np.ndarray        # yhat - m of the step
    info: SolveInfo
    rel_change: float
    S: Optional[np.ndarray] = None   # action buffer S and T = K S after the step
    T: Optional[np.ndarray] = None


def iterncgp(apply_K: Apply, y: np.ndarray, C: int, steps: int,
             policy: str = "cg", j_max: int = 100, rank_limit: Optional[int] = None,
             recycle: bool = True, tol_abs: float = 1e-5, tol_rel: float = 1e-5,
             outer_tol: Optional[float] = None,
             user_actions: Optional[List[np.ndarray]] = None,
             F0: Optional[np.ndarray] = None):
    """Algorithm 1 for the softmax likelihood with m = 0 and f_0 = m.

    ``apply_K`` applies the NC x NC prior covariance to CN-ordered vectors or
    (NC, b) matrices.  Returns the list of NewtonRecord, one per step.
    """
    N = len(y)
    n = N * C
    F = np.zeros((N, C)) if F0 is None else np.array(F0, dtype=np.float64)
    S, T = np.zeros((n, 0)), np.zeros((n, 0))
    recs = []
    for i in range(steps):
        Wp = lik.softmax_hessian_pinv_blocks(F)
        apply_Winv = (lambda Wp_: (lambda V: lik.apply_blocks(Wp_, V)))(Wp)
        rhs = pseudo_target_offset(F, y)                  # yhat(f_i) - m
        ua = None if user_actions is None else user_actions[i]
        v, Q, S, T, info = itergp(apply_K, apply_Winv, rhs, S, T, policy, j_max,
                                  tol_abs, tol_rel, rank_limit,
                                  recycle and policy != "unit", ua)
        F_new = apply_K(v).reshape(N, C)                  # f_{i+1} = K v + m
        g_old, g_new = F.reshape(-1), F_new.reshape(-1)
        nn = float(np.linalg.norm(g_new))
        rel = float(np.linalg.norm(g_new - g_old) / nn) if nn > 0 else float("inf")
        recs.append(NewtonRecord(F_new, v, Q, rhs, info, rel, S, T))
        F = F_new
        if outer_tol is not None and rel <= outer_tol:
            break
    return recs


def diag_likelihood_terms(name: str, f: np.ndarray, y: np.ndarray, noise_var: float = 1.0):
    """Gradient and diagonal of W(f)^{-1} of a likelihood whose negative
    Hessian is diagonal.

    poisson  (log link; appendix on the Poisson log likelihood):
             grad = y - exp(f), W^{-1} = diag(exp(-f))
    gaussian (observation variance noise_var; the conjugate case):
             grad = (y - f) / noise_var, W^{-1} = noise_var I
    """
    f = np.asarray(f, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if name == "poisson":
        return lik.poisson_grad(f, y), lik.poisson_winv_diag(f)
    if name == "gaussian":
        return (y - f) / noise_var, np.full(f.shape, float(noise_var))
    raise ValueError(f"unknown likelihood {name!r}")


def iterncgp_diag(apply_K: Apply, y: np.ndarray, steps: int, likelihood: str = "poisson",
                  noise_var: float = 1.0, policy: str = "cg", j_max: int = 100,
                  rank_limit: Optional[int] = None, recycle: bool = True,
                  tol_abs: float = 1e-5, tol_rel: float = 1e-5,
                  outer_tol: Optional[float] = None,
                  user_actions: Optional[List[np.ndarray]] = None,
                  f0: Optional[np.ndarray] = None):
    """Algorithm 1 for a likelihood with diagonal W^{-1} (Poisson, Gaussian),
    m = 0, f_0 = m.  y and f are vectors of length n (n = N for one latent
    function; n = N C CN-ordered for C independent ones).  The pseudo-targets
    are yhat - m = f + W^{-1} grad (the Newton step of section 3.1 written as
    a GP regression problem); IterGP (Algorithm 2) solves (K + W^{-1}) v =
    yhat - m with the recycled buffers (Algorithm 3); f_{i+1} = K v.
    Returns the list of NewtonRecord (F holds f as an (n, 1) array)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    f = np.zeros(n) if f0 is None else np.array(f0, dtype=np.float64)
    S, T = np.zeros((n, 0)), np.zeros((n, 0))
    recs = []
    for i in range(steps):
        grad, wd = diag_likelihood_terms(likelihood, f, y, noise_var)
        apply_Winv = (lambda wd_: (lambda V: (wd_[:, None] * V) if V.ndim == 2 else wd_ * V))(wd)
        rhs = f + wd * grad
        ua = None if user_actions is None else user_actions[i]
        v, Q, S, T, info = itergp(apply_K, apply_Winv, rhs, S, T, policy, j_max,
                                  tol_abs, tol_rel, rank_limit,
                                  recycle and policy != "unit", ua)
        f_new = apply_K(v)
        nn = float(np.linalg.norm(f_new))
        rel = float(np.linalg.norm(f_new - f) / nn) if nn > 0 else float("inf")
        recs.append(NewtonRecord(f_new[:, None], v, Q, rhs, info, rel, S, T))
        f = f_new
        if outer_tol is not None and rel <= outer_tol:
            break
    return recs


def iterncgp_block(apply_K: Apply, terms: Callable, N: int, C: int, steps: int,
                   policy: str = "cg", j_max: int = 100, rank_limit: Optional[int] = None,
                   recycle: bool = True, tol_abs: float = 1e-5, tol_rel: float = 1e-5,
                   outer_tol: Optional[float] = None,
                   user_actions: Optional[List[np.ndarray]] = None,
                   F0: Optional[np.ndarray] = None):
    """Algorithm 1 for a likelihood that factorises over the N points, m = 0,
    f_0 = m.  ``terms(F)`` returns the gradient of log p at F, shape (N, C),
    and the negative-Hessian blocks W_n, shape (N, C, C), each symmetric
    positive definite.  The Newton step of section 3.1 as GP regression:
    yhat - m = f + W^{-1} grad, then (K + W^{-1}) v = yhat - m by IterGP with
    W^{-1} block diagonal (each block inverted by numpy.linalg.inv),
    f_{i+1} = K v.  Returns the list of NewtonRecord."""
    n = N * C
    F = np.zeros((N, C)) if F0 is None else np.array(F0, dtype=np.float64)
    S, T = np.zeros((n, 0)), np.zeros((n, 0))
    recs = []
    for i in range(steps):
        grad, W = terms(F)
        Winv = np.linalg.inv(np.asarray(W, dtype=np.float64))
        apply_Winv = (lambda B: (lambda V: lik.apply_blocks(B, V)))(Winv)
        rhs = F.reshape(-1) + lik.apply_blocks(Winv, np.asarray(grad, dtype=np.float64).reshape(-1))
        ua = None if user_actions is None else user_actions[i]
        v, Q, S, T, info = itergp(apply_K, apply_Winv, rhs, S, T, policy, j_max,
                                  tol_abs, tol_rel, rank_limit,
                                  recycle and policy != "unit", ua)
        F_new = apply_K(v).reshape(N, C)
        g_old, g_new = F.reshape(-1), F_new.reshape(-1)
        nn = float(np.linalg.norm(g_new))
        rel = float(np.linalg.norm(g_new - g_old) / nn) if nn > 0 else float("inf")
        recs.append(NewtonRecord(F_new, v, Q, rhs, info, rel, S, T))
        F = F_new
        if outer_tol is not None and rel <= outer_tol:
            break
    return recs


def itergp_diag_noise(apply_K: Apply, winv_diag: np.ndarray, rhs: np.ndarray,
                      S: np.ndarray, T: np.ndarray, **kw):
    """Algorithm 2 for a diagonal observation noise W^{-1} (Poisson, Gaussian)."""
    return itergp(apply_K, lambda V: (winv_diag[:, None] * V) if V.ndim == 2 else winv_diag * V,
                  rhs, S, T, **kw)
