"""GPU parity of the IterNCGP path (itergp_init / itergp_newton_step /
itergp_predict) against the FP64 oracle.

* FP64, unit-vector policy at full budget (j_max = NC): every Newton iterate
  equals the exact Newton step (dense Cholesky), relative error <= 1e-9.
* FP64, the oracle's CG actions replayed (policy USER): iterates, representer
  weights and C_j = Q Q^T within 1e-10.
* FP64, free-running CG with recycling: same iteration counts, iterates
  within 1e-5; prediction kernels within 1e-10 of the oracle on the same state.
* FP32 with the oracle's own actions replayed (policy USER): the iterates and
  the predictive mean stay within 1e-4 relative of the FP64 oracle.
Every case runs with the residual formed by a fresh product with K (as the
algorithm is printed) and with K v carried by the K Q recurrence.
"""
import numpy as np
import pytest
import torch

import datagen
from oracle import itergp as oi
from oracle import kernels as ok
from oracle import newton as on
from oracle import predict as op
from paper_2310_20285_amd import api

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def cfg1():
    return datagen.config1()


def _model(w, X, **kw):
    dt = torch.float64 if kw.get("precision", "fp32") == "fp64" else torch.float32
    Xd = torch.tensor(X, dtype=dt, device="cuda")
    yd = torch.tensor(w.y, dtype=torch.int32, device="cuda")
    return api.IterNCGP(Xd, yd, w.C, w.kernel, w.lengthscale, w.outputscale, **kw), dt


RESIDUAL = pytest.mark.parametrize("residual", ["explicit", "recurrence"])


@RESIDUAL
def test_config1_unit_full_budget_is_exact_newton(gpu_lib, cfg1, residual):
    w = cfg1
    n = w.N * w.C
    m, dt = _model(w, w.X, policy="unit", j_max=n, recycle=False, tol_abs=0.0, tol_rel=0.0,
                   precision="fp64", max_buffer=n, residual_mode=residual)
    Kf = ok.full_kernel_cn(ok.kernel_matrix(w.X, w.X, w.kernel, w.lengthscale, w.outputscale), w.C)
    Fs, vs = on.exact_newton(Kf, w.y, w.C, 5)
    for i in range(5):
        info = m.newton_step()
        assert info["iters"] == n
        F = m.view(0).cpu().numpy().reshape(w.N, w.C)
        assert _rel(F, Fs[i + 1]) <= 1e-9, (i, _rel(F, Fs[i + 1]))
    v = m.view(1).cpu().numpy()
    assert _rel(v, vs[-1]) <= 1e-8


@RESIDUAL
def test_config1_fp64_user_replay_matches_oracle(gpu_lib, cfg1, residual):
    """The oracle's CG actions replayed through the GPU path (FP64): with the
    actions fixed, every remaining operation is a fixed linear-algebra
    pipeline, reproducible to ~1e-15 between rounding orders on the CPU."""
    w = cfg1
    kw = dict(j_max=60, rank_limit=40, recycle=True, tol_abs=1e-5, tol_rel=1e-5)
    Kf = ok.full_kernel_cn(ok.kernel_matrix(w.X, w.X, w.kernel, w.lengthscale, w.outputscale), w.C)
    recs = oi.iterncgp(lambda V: Kf @ V, w.y, w.C, 4, policy="cg", **kw)
    m, dt = _model(w, w.X, policy="user", precision="fp64", max_buffer=100,
                   residual_mode=residual, **kw)
    for i, rec in enumerate(recs):
        m.set_user_actions(torch.tensor(np.stack(rec.info.actions), dtype=dt, device="cuda"))
        info = m.newton_step()
        assert info["iters"] == rec.info.iters
        assert info["recycled_cols"] == (rec.info.vsr.eigvals.size if rec.info.vsr else 0)
        F = m.view(0).cpu().numpy().reshape(w.N, w.C)
        assert _rel(F, rec.F) <= 1e-10, (i, _rel(F, rec.F))
        assert _rel(m.view(1).cpu().numpy(), rec.v) <= 1e-10
        # C_j = Q Q^T is unique (Q itself is up to an orthogonal factor)
        Q = m.view(2).cpu().numpy().T
        z = np.random.default_rng(i).standard_normal(Q.shape[0])
        assert _rel(Q @ (Q.T @ z), rec.Q @ (rec.Q.T @ z)) <= 1e-9


@RESIDUAL
def test_config1_cg_recycling_free_running(gpu_lib, cfg1, residual):
    """Free-running CG in FP64 against the oracle.  The CG iterate itself is
    sensitive to rounding order here (two FP64 oracle runs that differ only in
    how K v is summed move F by ~1e-7 after 15 iterations: rounding excites the
    class-sum directions that W^+ annihilates), so the bar is the iteration
    count plus the 1e-5 predictive-level tolerance.  The prediction kernels
    are checked tightly against the oracle evaluated on the GPU's own v, Q."""
    w = cfg1
    kw = dict(policy="cg", j_max=60, rank_limit=40, recycle=True, tol_abs=1e-5, tol_rel=1e-5)
    m, dt = _model(w, w.X, precision="fp64", max_buffer=100, residual_mode=residual, **kw)
    Kf = ok.full_kernel_cn(ok.kernel_matrix(w.X, w.X, w.kernel, w.lengthscale, w.outputscale), w.C)
    recs = oi.iterncgp(lambda V: Kf @ V, w.y, w.C, 4, **kw)
    for i, rec in enumerate(recs):
        info = m.newton_step()
        assert info["iters"] == rec.info.iters, (i, info, rec.info.iters)
        F = m.view(0).cpu().numpy().reshape(w.N, w.C)
        assert _rel(F, rec.F) <= 1e-5, (i, _rel(F, rec.F))
    Xs = torch.tensor(w.Xs, dtype=dt, device="cuda")
    mean, var, probs = m.predict(Xs)
    v = m.view(1).cpu().numpy()
    Q = m.view(2).cpu().numpy().T
    mown = op.predictive_mean(w.Xs, w.X, v, w.C, w.kernel, w.lengthscale, w.outputscale)
    vown = op.predictive_var_root(w.Xs, w.X, Q, w.C, w.kernel, w.lengthscale, w.outputscale)
    assert _rel(mean.cpu().numpy(), mown) <= 1e-12
    np.testing.assert_allclose(var.cpu().numpy(), vown, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(probs.cpu().numpy(), op.probit_probs(mown, vown), rtol=1e-10,
                               atol=1e-13)
    mref = op.predictive_mean(w.Xs, w.X, recs[-1].v, w.C, w.kernel, w.lengthscale, w.outputscale)
    assert _rel(mean.cpu().numpy(), mref) <= 1e-5
    assert np.all(var.cpu().numpy() <= w.outputscale + 1e-12)


@RESIDUAL
def test_fp32_user_replay_matches_fp64_oracle(gpu_lib, residual):
    w = datagen.config2(N=1500, Ns=300)
    n = w.N * w.C
    KX = ok.kernel_matrix(w.X, w.X, w.kernel, w.lengthscale, w.outputscale)
    aK = lambda V: ok.apply_full_kernel_cn(KX, V, w.C)
    steps, jmax, R = 3, 40, 30
    recs = oi.iterncgp(aK, w.y, w.C, steps, policy="cg", j_max=jmax, rank_limit=R,
                       recycle=True, tol_abs=1e-5, tol_rel=1e-5)
    m, dt = _model(w, w.X, policy="user", j_max=jmax, rank_limit=R, recycle=True,
                   tol_abs=1e-5, tol_rel=1e-5, precision="fp32", max_buffer=jmax + R,
                   residual_mode=residual)
    for i, rec in enumerate(recs):
        acts = np.stack(rec.info.actions) if rec.info.actions else np.zeros((0, n))
        A = torch.tensor(acts, dtype=dt, device="cuda")
        m.set_user_actions(A)
        info = m.newton_step()
        F = m.view(0).cpu().numpy().reshape(w.N, w.C)
        assert _rel(F, rec.F) <= 1e-4, (i, _rel(F, rec.F), info)
    Xs = torch.tensor(w.Xs, dtype=dt, device="cuda")
    mean, var, _ = m.predict(Xs, probs=False)
    mref = op.predictive_mean(w.Xs, w.X, recs[-1].v, w.C, w.kernel, w.lengthscale, w.outputscale)
    assert _rel(mean.double().cpu().numpy(), mref) <= 1e-4


def test_step_in_parts_equals_whole_step(gpu_lib):
    """itergp_newton_step_begin / _iterate / _end give bitwise the iterates of
    itergp_newton_step; the order of the calls is enforced."""
    w = datagen.config2(N=1500, Ns=10)
    kw = dict(policy="cg", j_max=40, rank_limit=20, recycle=True, precision="fp32",
              residual_mode="recurrence")
    a, _ = _model(w, w.X, **kw)
    b, _ = _model(w, w.X, **kw)
    from paper_2310_20285_amd._lib import IterGPError
    for step in range(3):
        ia = a.newton_step()
        b.step_begin()
        with pytest.raises(IterGPError):
            b.step_begin()
        with pytest.raises(IterGPError):
            b.compress(5)
        parts = 0
        while not b.step_iterate(3):
            parts += 1
            if parts == 1:
                # the posterior at the current iteration is available mid-step
                mean, _, _ = b.predict(torch.tensor(w.Xs, dtype=torch.float32, device="cuda"),
                                       var=False, probs=False)
                assert torch.isfinite(mean).all()
        ib = b.step_end()
        with pytest.raises(IterGPError):
            b.step_end()
        assert ia["iters"] == ib["iters"]
        assert torch.equal(a.view(0), b.view(0)) and torch.equal(a.view(2), b.view(2))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("residual", ["explicit", "recurrence"])
def test_free_running_cg_repeatable(gpu_lib, cfg1, prec, residual):
    """The solver enqueues iterations ahead of their convergence test and a
    device gate stops the ones past it: three fresh fits give bitwise the same
    iteration counts, buffers and iterates (the gate and the scalars the
    iteration kernels read must never be read stale)."""
    w = cfg1
    kw = dict(policy="cg", j_max=60, rank_limit=40, recycle=True, tol_abs=1e-5, tol_rel=1e-5)
    runs = []
    for _ in range(3):
        m, _ = _model(w, w.X, precision=prec, max_buffer=100, residual_mode=residual, **kw)
        infos = [m.newton_step() for _ in range(4)]
        runs.append(([(i["iters"], i["buffer_cols"], i["converged"]) for i in infos],
                     m.view(0).clone(), m.view(2).clone()))
    for r in runs[1:]:
        assert r[0] == runs[0][0]
        assert torch.equal(r[1], runs[0][1]) and torch.equal(r[2], runs[0][2])


def test_window_boundaries_match_single_iterations(gpu_lib):
    """Slices of 1..5 iterations (windows cut at every size) give bitwise the
    iterates of the whole step."""
    w = datagen.config2(N=1200, Ns=10)
    kw = dict(policy="cg", j_max=23, rank_limit=20, recycle=True, precision="fp32",
              residual_mode="recurrence")
    ref, _ = _model(w, w.X, **kw)
    ir = [ref.newton_step() for _ in range(2)]
    for sl in (1, 2, 3, 5):
        m, _ = _model(w, w.X, **kw)
        for step in range(2):
            m.step_begin()
            while not m.step_iterate(sl):
                pass
            info = m.step_end()
            assert info["iters"] == ir[step]["iters"], (sl, step)
        assert torch.equal(m.view(0), ref.view(0)) and torch.equal(m.view(2), ref.view(2)), sl


def test_profiling_stride(gpu_lib, cfg1):
    """Product tracing: stride 1 times every product of the steps that ran,
    stride 3 a subset, with the same evaluations per timed product (the
    symmetric count n(n+1)/2); the iterates do not depend on tracing; a negative
    stride is refused."""
    w = cfg1
    kw = dict(policy="cg", j_max=30, rank_limit=20, recycle=True, precision="fp32",
              residual_mode="recurrence", max_buffer=90)
    out = {}
    for every in (1, 3):
        m, _ = _model(w, w.X, **kw)
        m.set_profiling(True, every=every)
        infos = [m.newton_step() for _ in range(3)]
        prof = m.profile()
        total = sum(i["k_products"] for i in infos)
        if every == 1:
            assert prof["kv_launches"] == total
        else:
            assert 1 <= prof["kv_launches"] < total
        assert prof["kv_evals"] / prof["kv_launches"] == pytest.approx(w.N * (w.N + 1) / 2)
        assert prof["kv_ms"] > 0.0 and prof["steps"] == 3
        out[every] = m.view(0).double().cpu().numpy()
    assert np.array_equal(out[1], out[3])
    with pytest.raises(Exception):
        m.set_profiling(True, every=-1)
