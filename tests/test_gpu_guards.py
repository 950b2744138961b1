"""The solver's guard paths on the GPU against the FP64 oracle.

* Breakdown (the stopping-criteria appendix ends the solve when eta_j <= 0):
  a zero action among the user actions gives eta = 0 exactly on both sides.
  The step ends there and the action and its product are not kept.  The zero
  action sits inside a window of iterations enqueued ahead of their
  convergence test (3rd action) or at a window's start (5th).  The next step
  recycles the kept columns.  Checked: iteration count, the breakdown flag,
  buffer and recycled column counts, f, v and C_j = Q Q^T (FP64, both residual
  modes); the batched step against single-model steps with the same actions
  (FP32).
* Eigenvalue floor of the virtual solver run (Algorithm 3; eigenpairs with
  lambda <= lambda_max B eps_64 are dropped before Lambda^{-1/2}): one action
  of a 250-action step is a near copy of another (offset 5e-7).  Its Schur
  complement eta is clearly positive (about 90 eps lambda_max), so it is
  accepted in the step.  In the next step's M its eigenvalue is about 37x
  below the floor, so it is dropped on both sides.  The test first checks
  these margins on the oracle's own numbers.
* Psi (the log posterior at the new iterate, log p(y|f) - g^T v / 2) against
  oracle.newton.psi_from_v.
* Status codes through the C ABI: IGP_ENOMEM for an arena shorter than
  itergp_state_bytes (before any device work) and IGP_EINVAL for a NaN in X
  or a label outside [0, C).
"""
import ctypes as ct

import numpy as np
import pytest
import torch

import datagen
from oracle import itergp as oi
from oracle import kernels as ok
from oracle import likelihood as lik
from oracle import newton as on
from paper_2310_20285_amd import _lib as L
from paper_2310_20285_amd import api

pytestmark = pytest.mark.gpu
EPS64 = float(np.finfo(np.float64).eps)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def small():
    w = datagen.gp_classification(7, 100, 4, 3, "matern32", 1.0, 1.0, Ns=10)
    Kf = ok.full_kernel_cn(ok.kernel_matrix(w.X, w.X, w.kernel, w.lengthscale,
                                            w.outputscale), w.C)
    return w, Kf


def _model(w, dt, **kw):
    X = torch.tensor(w.X, dtype=dt, device="cuda")
    y = torch.tensor(w.y, dtype=torch.int32, device="cuda")
    return api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="user",
                        recycle=True, tol_abs=0.0, tol_rel=0.0, **kw)


def _actions(n, k, seed, zero_at=None):
    A = np.random.default_rng(seed).standard_normal((n, k))
    if zero_at is not None:
        A[:, zero_at] = 0.0
    return A


@pytest.mark.parametrize("residual", ["explicit", "recurrence"])
@pytest.mark.parametrize("zero_at", [2, 4])
def test_breakdown_zero_action_matches_oracle(gpu_lib, small, residual, zero_at):
    w, Kf = small
    n = w.N * w.C
    A1 = _actions(n, 8, 11, zero_at)
    A2 = _actions(n, 4, 12)
    recs = oi.iterncgp(lambda V: Kf @ V, w.y, w.C, 2, policy="user", j_max=8, rank_limit=None,
                       recycle=True, tol_abs=0.0, tol_rel=0.0, user_actions=[A1, A2])
    assert recs[0].info.breakdown and recs[0].info.iters == zero_at
    m = _model(w, torch.float64, j_max=8, rank_limit=-1, precision="fp64", max_buffer=16,
               residual_mode=residual)
    for A, rec in zip((A1, A2), recs):
        m.set_user_actions(torch.tensor(A.T.copy(), dtype=torch.float64, device="cuda"))
        info = m.newton_step()
        print(f"zero at {zero_at} ({residual}): {info}", flush=True)
        assert info["iters"] == rec.info.iters
        assert info["breakdown"] == int(rec.info.breakdown)
        assert info["buffer_cols"] == rec.S.shape[1]
        assert info["recycled_cols"] == (rec.info.vsr.eigvals.size if rec.info.vsr else 0)
        F = m.view(0).cpu().numpy().reshape(w.N, w.C)
        assert _rel(F, rec.F) <= 1e-10
        assert _rel(m.view(1).cpu().numpy(), rec.v) <= 1e-10
        Q = m.view(2).cpu().numpy().T
        assert _rel(Q @ Q.T, rec.Q @ rec.Q.T) <= 1e-10


@pytest.mark.parametrize("device_control", [
    False,
    pytest.param(True, marks=pytest.mark.skip(reason=("a run of this test hung with a variant of the persistent product kernels that skipped the tiles of stopped problems (since removed); the cause has not been found, so device-controlled batched steps stay off the GPU until it is"))),
])
def test_breakdown_in_batched_step_matches_single(gpu_lib, small, device_control):
    """FP32, recurrence residual: a batch of three models, one with a zero
    action at the 3rd position, one at the 5th, one without, against the same
    models stepped one at a time with the same actions; with device control
    the breakdowns fall inside a window of iterations."""
    w, _ = small
    n = w.N * w.C
    zeros = [2, 4, None]
    acts = [[_actions(n, 8, 21 + k, z), _actions(n, 4, 31 + k)] for k, z in enumerate(zeros)]
    kw = dict(j_max=8, rank_limit=-1, precision="fp32", max_buffer=16,
              residual_mode="recurrence")
    batch = [_model(w, torch.float32, **kw) for _ in zeros]
    single = [_model(w, torch.float32, **kw) for _ in zeros]
    buf = None
    for step in range(2):
        for mb, ms, a in zip(batch, single, acts):
            for m in (mb, ms):
                m.set_user_actions(torch.tensor(a[step].T.copy(), dtype=torch.float32,
                                                device="cuda"))
        infos, buf = api.newton_step_batched(batch, buf, device_control=device_control)
        for k, (mb, ms) in enumerate(zip(batch, single)):
            si = ms.newton_step()
            bi = infos[k]
            print(f"step {step + 1} model {k}: batched {bi['iters']}/{bi['breakdown']}/"
                  f"{bi['buffer_cols']}, single {si['iters']}/{si['breakdown']}/"
                  f"{si['buffer_cols']}", flush=True)
            for key in ("iters", "breakdown", "buffer_cols", "recycled_cols"):
                assert bi[key] == si[key], (step, k, key)
            Fb = mb.view(0).double().cpu().numpy()
            Fs = ms.view(0).double().cpu().numpy()
            assert _rel(Fb, Fs) <= 1e-5
    assert [i["breakdown"] for i in infos] == [0, 0, 0]


def test_eigenvalue_floor_matches_oracle(gpu_lib, small):
    w, Kf = small
    n = w.N * w.C
    rng = np.random.default_rng(3)
    B1 = 250
    A1 = rng.standard_normal((n, B1))
    A1 /= np.linalg.norm(A1, axis=0)
    g = rng.standard_normal(n)
    g /= np.linalg.norm(g)
    a = A1[:, 0] + 5e-7 * g                      # near copy of the first action
    A1[:, 99] = a / np.linalg.norm(a)
    A2 = rng.standard_normal((n, 5))
    recs = oi.iterncgp(lambda V: Kf @ V, w.y, w.C, 2, policy="user", j_max=B1, rank_limit=None,
                       recycle=True, tol_abs=0.0, tol_rel=0.0, user_actions=[A1, A2])
    # margins on the oracle's own numbers: the near copy is accepted in step 1
    # (eta well above rounding) and its eigenvalue in step 2's M is well below
    # the floor, all others well above
    r0 = recs[0]
    assert r0.info.iters == B1 and not r0.info.breakdown
    S, T = r0.S, r0.T
    M = S.T @ (T + lik.apply_blocks(lik.softmax_hessian_pinv_blocks(r0.F), S))
    lam = np.sort(np.linalg.eigvalsh(0.5 * (M + M.T)))[::-1]
    floor = lam[0] * B1 * EPS64
    assert r0.info.etas[99] >= 30 * EPS64 * lam[0]
    assert abs(lam[-1]) <= floor / 10 and lam[-2] >= 1e3 * floor
    assert recs[1].info.vsr.n_dropped_floor == 1

    m = _model(w, torch.float64, j_max=B1, rank_limit=-1, precision="fp64", max_buffer=B1 + 8,
               residual_mode="recurrence")
    for A, rec in zip((A1, A2), recs):
        m.set_user_actions(torch.tensor(A.T.copy(), dtype=torch.float64, device="cuda"))
        info = m.newton_step()
        print(f"floor test: {info}", flush=True)
        assert info["iters"] == rec.info.iters
        dropped = rec.info.vsr.n_dropped_floor if rec.info.vsr else 0
        assert info["eig_dropped"] == dropped
        assert info["recycled_cols"] == (rec.info.vsr.eigvals.size if rec.info.vsr else 0)
        F = m.view(0).cpu().numpy().reshape(w.N, w.C)
        assert _rel(F, rec.F) <= 1e-6


def test_psi_matches_oracle(gpu_lib, small):
    """Psi after each Newton step of a replayed CG fit (FP64) against the
    oracle's log posterior at the same iterate and weights."""
    w, Kf = small
    recs = oi.iterncgp(lambda V: Kf @ V, w.y, w.C, 3, policy="cg", j_max=30, rank_limit=20,
                       recycle=True)
    m = _model(w, torch.float64, j_max=30, rank_limit=20, precision="fp64", max_buffer=60,
               residual_mode="explicit")
    for rec in recs:
        m.set_user_actions(torch.tensor(np.stack(rec.info.actions), dtype=torch.float64,
                                        device="cuda"))
        info = m.newton_step()
        ref = on.psi_from_v(rec.F, w.y, rec.v)
        print(f"psi {info['psi']:.12f} oracle {ref:.12f}", flush=True)
        assert abs(info["psi"] - ref) <= 1e-9 * abs(ref)


def _init(lib, X, y, N, D, C, arena, nbytes, cfg):
    kp, n_kp = api.kernel_params("matern32", 1.0, 1.0)
    h = ct.c_void_p()
    rc = lib.itergp_init(ct.byref(h), kp, n_kp, ct.byref(cfg), ct.c_void_p(X.data_ptr()),
                         ct.c_void_p(y.data_ptr()), N, D, C, ct.c_void_p(arena.data_ptr()),
                         nbytes, ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, h


def test_status_codes_through_the_abi(gpu_lib, small):
    w, _ = small
    lib = L.load()
    cfg = api.solver_config(policy="cg", j_max=10, rank_limit=5, precision="fp32",
                            max_buffer=15)
    N, D, C = w.N, w.X.shape[1], w.C
    need = lib.itergp_state_bytes(N, D, C, ct.byref(cfg))
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
    y = torch.tensor(w.y, dtype=torch.int32, device="cuda")
    # an arena one byte short
    rc, h = _init(lib, X, y, N, D, C, arena, need - 1, cfg)
    assert rc == L.IGP_ENOMEM and not h.value
    assert b"arena too small" in lib.igp_last_error()
    # a NaN in X
    Xn = X.clone()
    Xn[17, 2] = float("nan")
    rc, h = _init(lib, Xn, y, N, D, C, arena, need, cfg)
    assert rc == L.IGP_EINVAL and not h.value
    assert b"non-finite entries in X" in lib.igp_last_error()
    # a label outside [0, C)
    yb = y.clone()
    yb[5] = C
    rc, h = _init(lib, X, yb, N, D, C, arena, need, cfg)
    assert rc == L.IGP_EINVAL and not h.value
    # the valid call succeeds on the same arena
    rc, h = _init(lib, X, y, N, D, C, arena, need, cfg)
    assert rc == L.IGP_OK and h.value
    assert lib.itergp_destroy(h) == L.IGP_OK
