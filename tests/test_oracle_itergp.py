"""Pins for oracle.itergp (Algorithms 1-3) against facts the paper and
textbook linear algebra fix."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import itergp as oi
from oracle import kernels as ok
from oracle import likelihood as lk
from oracle import newton as on


def _system(seed=0, N=8, C=3, D=2, kind="matern32", scale=1.0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, D))
    y = rng.integers(0, C, size=N)
    KX = ok.kernel_matrix(X, X, kind, 1.0, 1.0)
    Kf = ok.full_kernel_cn(KX, C)
    F = rng.standard_normal((N, C)) * scale
    Wp = lk.softmax_hessian_pinv_blocks(F)
    Khat = Kf + lk.dense_block_diag(Wp)
    rhs = on.pseudo_target_offset(F, y)
    aK = lambda V: Kf @ V
    aW = lambda V: lk.apply_blocks(Wp, V)
    return dict(Kf=Kf, Khat=Khat, rhs=rhs, aK=aK, aW=aW, F=F, y=y, C=C, KX=KX, X=X)


def _empty(n):
    return np.zeros((n, 0)), np.zeros((n, 0))


def test_full_budget_unit_policy_is_exact_solve():
    s = _system()
    n = s["rhs"].size
    v, Q, S, T, info = oi.itergp(s["aK"], s["aW"], s["rhs"], *_empty(n), policy="unit",
                                 j_max=n, recycle=False, tol_abs=0, tol_rel=0)
    assert info.iters == n
    np.testing.assert_allclose(v, np.linalg.solve(s["Khat"], s["rhs"]), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(Q @ Q.T, np.linalg.inv(s["Khat"]), rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("j", [1, 4, 11])
def test_unit_policy_equals_leading_block_solve(j):
    s = _system(1)
    n = s["rhs"].size
    v, *_ = oi.itergp(s["aK"], s["aW"], s["rhs"], *_empty(n), policy="unit", j_max=j,
                      recycle=False, tol_abs=0, tol_rel=0)
    ref = np.zeros(n)
    ref[:j] = np.linalg.solve(s["Khat"][:j, :j], s["rhs"][:j])
    np.testing.assert_allclose(v, ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("j", [1, 3, 6])
def test_cg_policy_equals_textbook_cg(j):
    s = _system(2)
    n = s["rhs"].size
    v, *_ = oi.itergp(s["aK"], s["aW"], s["rhs"], *_empty(n), policy="cg", j_max=j,
                      recycle=False, tol_abs=0, tol_rel=0)
    x, _ = spla.cg(s["Khat"], s["rhs"], x0=np.zeros(n), maxiter=j, rtol=1e-300, atol=0.0)
    np.testing.assert_allclose(v, x, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("j", [2, 5, 9])
def test_precision_root_equals_projected_inverse(j):
    s = _system(3)
    n = s["rhs"].size
    v, Q, S, T, info = oi.itergp(s["aK"], s["aW"], s["rhs"], *_empty(n), policy="cg",
                                 j_max=j, recycle=False, tol_abs=0, tol_rel=0)
    Cj = S @ np.linalg.solve(S.T @ s["Khat"] @ S, S.T)
    np.testing.assert_allclose(Q @ Q.T, Cj, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(v, Cj @ s["rhs"], rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(T, s["Kf"] @ S, atol=1e-13)
    r = s["rhs"] - s["Khat"] @ v
    np.testing.assert_allclose(S.T @ r, 0.0, atol=1e-10 * np.linalg.norm(s["rhs"]))


def test_action_scale_invariance():
    s = _system(4)
    n = s["rhs"].size
    a = oi.itergp(s["aK"], s["aW"], s["rhs"], *_empty(n), policy="cg", j_max=7,
                  recycle=False, tol_abs=0, tol_rel=0, normalize_actions=True)
    b = oi.itergp(s["aK"], s["aW"], s["rhs"], *_empty(n), policy="cg", j_max=7,
                  recycle=False, tol_abs=0, tol_rel=0, normalize_actions=False)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(a[1] @ a[1].T, b[1] @ b[1].T, rtol=1e-8, atol=1e-10)


def test_virtual_solver_run_properties():
    # buffers from a run on problem A, recycled on problem B (new W)
    sa = _system(5, scale=1.0)
    n = sa["rhs"].size
    _, _, S, T, _ = oi.itergp(sa["aK"], sa["aW"], sa["rhs"], *_empty(n), policy="cg",
                              j_max=6, recycle=False, tol_abs=0, tol_rel=0)
    rng = np.random.default_rng(6)
    F2 = sa["F"] + 0.3 * rng.standard_normal(sa["F"].shape)
    Wp2 = lk.softmax_hessian_pinv_blocks(F2)
    aW2 = lambda V: lk.apply_blocks(Wp2, V)
    Khat2 = sa["Kf"] + lk.dense_block_diag(Wp2)
    rhs2 = on.pseudo_target_offset(F2, sa["y"])
    Q0, S2, T2, vinfo = oi.virtual_solver_run(S, T, aW2)
    v0 = Q0 @ (Q0.T @ rhs2)
    # C_0 = S (S^T Khat S)^{-1} S^T
    C0 = S @ np.linalg.solve(S.T @ Khat2 @ S, S.T)
    np.testing.assert_allclose(Q0 @ Q0.T, C0, rtol=1e-7, atol=1e-9)
    # Proposition: residual in span{S} is zero
    r0 = rhs2 - Khat2 @ v0
    np.testing.assert_allclose(S.T @ r0, 0.0, atol=1e-10 * np.linalg.norm(rhs2))
    # Proposition: Khat-projected error in span{S} is zero
    vstar = np.linalg.solve(Khat2, rhs2)
    np.testing.assert_allclose(C0 @ Khat2 @ (vstar - v0), 0.0, atol=1e-9)
    # re-weighted buffers: T2 = K S2 and M~ = Lambda
    np.testing.assert_allclose(T2, sa["Kf"] @ S2, atol=1e-12)
    np.testing.assert_allclose(S2.T @ Khat2 @ S2, np.diag(vinfo.eigvals), atol=1e-9)


def test_compression_keeps_largest_eigenpairs_and_r0_gives_zero():
    s = _system(7)
    n = s["rhs"].size
    _, _, S, T, _ = oi.itergp(s["aK"], s["aW"], s["rhs"], *_empty(n), policy="cg",
                              j_max=8, recycle=False, tol_abs=0, tol_rel=0)
    M = S.T @ (T + s["aW"](S))
    lam_all = np.sort(np.linalg.eigvalsh(0.5 * (M + M.T)))[::-1]
    Q0, S3, T3, info = oi.virtual_solver_run(S, T, s["aW"], rank_limit=3)
    np.testing.assert_allclose(info.eigvals, lam_all[:3], rtol=1e-12)
    assert S3.shape[1] == 3 and info.n_dropped_rank == 5
    Qz, Sz, Tz, infz = oi.virtual_solver_run(S, T, s["aW"], rank_limit=0)
    assert Qz.shape[1] == 0
    v, *_ = oi.itergp(s["aK"], s["aW"], s["rhs"], S, T, policy="cg", j_max=0, rank_limit=0)
    assert np.all(v == 0.0)


def test_full_rank_recycling_is_exact_at_j0():
    s = _system(8)
    n = s["rhs"].size
    _, _, S, T, _ = oi.itergp(s["aK"], s["aW"], s["rhs"], *_empty(n), policy="unit",
                              j_max=n, recycle=False, tol_abs=0, tol_rel=0)
    v, *_ = oi.itergp(s["aK"], s["aW"], s["rhs"], S, T, policy="cg", j_max=0)
    np.testing.assert_allclose(v, np.linalg.solve(s["Khat"], s["rhs"]), rtol=1e-8, atol=1e-10)


def test_trace_identity_for_eigenvector_actions():
    # Proposition "Total Marginal Uncertainty": W^{-1} = 0, S = eigenvectors of K
    s = _system(9)
    Kf = s["Kf"]
    lam, B = np.linalg.eigh(Kf)
    S = B[:, -5:]
    T = Kf @ S
    Q0, S2, T2, info = oi.virtual_solver_run(S, T, lambda V: 0.0 * V)
    C0 = Q0 @ Q0.T
    tr_post = np.trace(Kf) - np.trace(Kf @ C0 @ Kf)
    M = S.T @ T
    np.testing.assert_allclose(tr_post, np.trace(Kf) - np.trace(M), rtol=1e-10)
    np.testing.assert_allclose(tr_post, lam[:-5].sum(), rtol=1e-10)


def test_breakdown_pops_the_action():
    s = _system(10)
    n = s["rhs"].size
    ua = np.zeros((n, 3))
    ua[0, 0] = 1.0          # e_1, then a zero action (eta = 0 -> breakdown)
    v, Q, S, T, info = oi.itergp(s["aK"], s["aW"], s["rhs"], *_empty(n), policy="user",
                                 j_max=3, recycle=False, tol_abs=0, tol_rel=0, user_actions=ua)
    assert info.breakdown and info.iters == 1
    assert S.shape[1] == 1 and T.shape[1] == 1 and Q.shape[1] == 1


def test_iterncgp_full_budget_unit_matches_exact_newton():
    rng = np.random.default_rng(11)
    N, C = 9, 3
    X = rng.standard_normal((N, 2))
    y = rng.integers(0, C, size=N)
    Kf = ok.full_kernel_cn(ok.kernel_matrix(X, X, "matern32", 1.0, 1.0), C)
    recs = oi.iterncgp(lambda V: Kf @ V, y, C, 5, policy="unit", j_max=N * C,
                       recycle=False, tol_abs=0, tol_rel=0)
    Fs, vs = on.exact_newton(Kf, y, C, 5)
    for rec, F, v in zip(recs, Fs[1:], vs):
        np.testing.assert_allclose(rec.F, F, rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(rec.v, v, rtol=1e-8, atol=1e-10)


def test_iterncgp_cg_with_recycling_matches_exact_newton():
    rng = np.random.default_rng(12)
    N, C = 10, 3
    X = rng.standard_normal((N, 2))
    y = rng.integers(0, C, size=N)
    Kf = ok.full_kernel_cn(ok.kernel_matrix(X, X, "matern32", 1.0, 1.0), C)
    recs = oi.iterncgp(lambda V: Kf @ V, y, C, 4, policy="cg", j_max=N * C,
                       recycle=True, tol_abs=1e-12, tol_rel=1e-12)
    Fs, _ = on.exact_newton(Kf, y, C, 4)
    for rec, F in zip(recs, Fs[1:]):
        np.testing.assert_allclose(rec.F, F, rtol=1e-7, atol=1e-8)
    # recycling: later steps need fewer new actions than the first
    assert recs[-1].info.iters < recs[0].info.iters
