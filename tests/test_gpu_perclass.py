"""One kernel per latent function (same family, class-specific lengthscale and
outputscale) on the GPU path, against the FP64 oracle:

* glm_kernel_matmul with n_kp = C: every entry within the product tolerance
  of the kernel tests (1e-12 FP64, 8 eps32 (8 + sqrt n2) FP32, relative to the
  per-class K|V|), over several tiles, ragged tails and all kernel families;
* IterNCGP with per-class kernels, the oracle's CG actions replayed: iterates
  within 1e-10 (FP64) / 1e-4 (FP32) of the oracle; prediction (mean and
  variance with the class-specific prior variances) within 1e-10 of the
  oracle's formulas on the GPU's own state;
* K(X, X) v with n_kp = C in FP32 (one vector, C <= 8): the symmetric
  matrix-core kernel's per-class form, element by element, over several
  super-blocks and ragged tails, within the first-order bound of the FP32
  norm expansion (the BF16 tests' bound with exact inputs):
    |got - ref| <= (os_c Lk / l_c^2) sum_m dr2_nm |v_m| + 8 eps32 (8 + sqrt n) (K_c|v|)
    dr2_nm = 4 sqrt(D) eps32 (|a_n|^2 + |a_m|^2)   (a: rows centred on the mean)
  Lk = max |dk/d(r^2)| / os: 1/2 (RBF), 3/2 (Matern-3/2), 5/6 (Matern-5/2).  Near
  r = 0 the expansion's absolute error in r^2 grows as 1/l^2, so the second
  term alone does not hold at short lengthscales (here down to 0.6);
* n_kp = C with equal parameters reproduces the shared-kernel result;
  BF16 with n_kp > 1 is refused, and so is a per-class model in a batched step.
"""
import math

import numpy as np
import pytest
import torch

import datagen
from datagen import KERNEL_KINDS
from oracle import itergp as oi
from oracle import kernels as ok
from oracle import predict as op
from paper_2310_20285_amd import api
from paper_2310_20285_amd._lib import IterGPError

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _params(C, seed):
    rng = np.random.default_rng(seed)
    return list(rng.uniform(0.6, 2.0, C)), list(rng.uniform(0.5, 1.8, C))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", KERNEL_KINDS)
@pytest.mark.parametrize("shape", [(200, 173, 3, 3, 1), (67, 300, 16, 5, 2), (1, 1, 1, 2, 1),
                                   (129, 700, 8, 4, 3)])
def test_per_class_kernel_matmul(gpu_lib, prec, kind, shape):
    n1, n2, d, C, nb = shape
    rng = np.random.default_rng(n1 * 7 + n2 + d + C)
    ells, oss = _params(C, n1 + C)
    dt = torch.float64 if prec == "fp64" else torch.float32
    X1 = torch.tensor(rng.standard_normal((n1, d)), dtype=dt, device="cuda")
    X2 = torch.tensor(rng.standard_normal((n2, d)), dtype=dt, device="cuda")
    V = torch.tensor(rng.standard_normal((nb, n2 * C)), dtype=dt, device="cuda")
    out = api.glm_kernel_matmul(X1, X2, V, C, kind, ells, oss, prec).double().cpu().numpy()
    X1h, X2h, Vh = (t.double().cpu().numpy() for t in (X1, X2, V))
    Ks = ok.kernel_matrices_per_class(X1h, X2h, kind, ells, oss)
    tol = 1e-12 if prec == "fp64" else 8 * EPS32 * (8 + math.sqrt(n2))
    for b in range(nb):
        ref = ok.apply_kernel_per_class(Ks, Vh[b])
        scale = ok.apply_kernel_per_class(Ks, np.abs(Vh[b]))
        err = np.abs(out[b] - ref)
        assert np.all(err <= tol * scale + 1e-300), (err / scale).max()


@pytest.mark.parametrize("kind", KERNEL_KINDS)
@pytest.mark.parametrize("n,d,C", [(1, 3, 2), (300, 16, 5), (1000, 8, 8), (2777, 16, 3),
                                   (4100, 32, 1)])
def test_per_class_symmetric_product(gpu_lib, kind, n, d, C):
    """The same point set on both sides and one vector: the symmetric
    matrix-core kernel's per-class form (Matern-1/2 keeps the direct-difference
    kernel)."""
    rng = np.random.default_rng(n + 31 * d + C)
    ells, oss = _params(C, n + d)
    X = torch.tensor(rng.standard_normal((n, d)), dtype=torch.float32, device="cuda")
    V = torch.tensor(rng.standard_normal(n * C), dtype=torch.float32, device="cuda")
    out = api.glm_kernel_matmul(X, X, V, C, kind, ells, oss, "fp32").double().cpu().numpy()
    Xh, Vh = X.double().cpu().numpy(), V.double().cpu().numpy()
    Ks = ok.kernel_matrices_per_class(Xh, Xh, kind, ells, oss)
    ref = ok.apply_kernel_per_class(Ks, Vh)
    scale = ok.apply_kernel_per_class(Ks, np.abs(Vh))
    A = Xh - Xh.mean(axis=0)
    na = (A * A).sum(1)
    va = np.abs(Vh).reshape(n, C)
    # sum_m dr2_nm |v_m| per class, with dr2_nm = 4 sqrt(D) eps32 (|a_n|^2 + |a_m|^2)
    ne = 4 * math.sqrt(d) * EPS32 * (na[:, None] * va.sum(0)[None, :] + (na @ va)[None, :])
    lk = {"rbf": 0.5, "matern32": 1.5, "matern52": 5.0 / 6.0}.get(kind, 0.0)
    ne *= np.array([o * lk / l ** 2 for l, o in zip(ells, oss)])[None, :]
    if kind == "matern12":      # the direct-difference kernel: no expansion term
        ne[:] = 0.0
    bound = ne.reshape(-1) + 8 * EPS32 * (8 + math.sqrt(n)) * scale
    err = np.abs(out - ref)
    assert np.all(err <= bound + 1e-300), (err / bound).max()


def test_per_class_model_refused_in_batched_step(gpu_lib):
    w = datagen.config4(seed=2, n_problems=1, n_lo=200, n_hi=300)[0]
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
    y = torch.tensor(w.y, dtype=torch.int32, device="cuda")
    ells, oss = _params(w.C, 3)
    m = api.IterNCGP(X, y, w.C, w.kernel, ells, oss, policy="cg", j_max=5, precision="fp32",
                     residual_mode="recurrence", max_buffer=10)
    with pytest.raises(IterGPError, match="one kernel shared"):
        api.newton_step_batched([m])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_equal_class_parameters_reproduce_shared_kernel(gpu_lib, prec, tol):
    rng = np.random.default_rng(4)
    dt = torch.float64 if prec == "fp64" else torch.float32
    X = torch.tensor(rng.standard_normal((300, 6)), dtype=dt, device="cuda")
    V = torch.tensor(rng.standard_normal(300 * 4), dtype=dt, device="cuda")
    shared = api.glm_kernel_matmul(X, X, V, 4, "matern52", 1.1, 0.9, prec).double().cpu().numpy()
    per = api.glm_kernel_matmul(X, X, V, 4, "matern52", [1.1] * 4, [0.9] * 4,
                                prec).double().cpu().numpy()
    assert _rel(per, shared) <= tol


def test_per_class_bf16_refused(gpu_lib):
    X = torch.zeros((10, 3), device="cuda")
    V = torch.zeros(20, device="cuda")
    with pytest.raises(IterGPError):
        api.glm_kernel_matmul(X, X, V, 2, "rbf", [1.0, 2.0], [1.0, 1.0], "bf16")


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
@pytest.mark.parametrize("residual", ["explicit", "recurrence"])
def test_per_class_newton_user_replay(gpu_lib, prec, tol, residual):
    w = datagen.gp_classification(31, 300, 3, 3, "matern32", 1.0, 1.0)
    ells, oss = [0.7, 1.2, 1.9], [0.6, 1.0, 1.5]
    Ks = ok.kernel_matrices_per_class(w.X, w.X, "matern32", ells, oss)
    Kf = ok.full_kernel_cn_per_class(Ks)
    kw = dict(j_max=40, rank_limit=25, recycle=True, tol_abs=1e-5, tol_rel=1e-5)
    recs = oi.iterncgp(lambda V: Kf @ V, w.y, w.C, 3, policy="cg", **kw)
    dt = torch.float64 if prec == "fp64" else torch.float32
    X = torch.tensor(w.X, dtype=dt, device="cuda")
    y = torch.tensor(w.y, dtype=torch.int32, device="cuda")
    m = api.IterNCGP(X, y, w.C, "matern32", ells, oss, policy="user", precision=prec,
                     max_buffer=65, residual_mode=residual, **kw)
    for rec in recs:
        m.set_user_actions(torch.tensor(np.stack(rec.info.actions), dtype=dt, device="cuda"))
        info = m.newton_step()
        assert info["iters"] == rec.info.iters
        assert _rel(m.view(0).double().cpu().numpy(), rec.F.reshape(-1)) <= tol
    Xs = np.random.default_rng(5).standard_normal((40, 3))
    mean, var, _ = m.predict(torch.tensor(Xs, dtype=dt, device="cuda"), probs=False)
    v = m.view(1).double().cpu().numpy()
    Q = m.view(2).double().cpu().numpy().T
    Xh = X.double().cpu().numpy()
    Xsh = torch.tensor(Xs, dtype=dt).double().numpy()
    mref = op.predictive_mean_per_class(Xsh, Xh, v, "matern32", ells, oss)
    vref = op.predictive_var_root_per_class(Xsh, Xh, Q, "matern32", ells, oss)
    ptol = 1e-10 if prec == "fp64" else 1e-4
    assert _rel(mean.double().cpu().numpy(), mref) <= ptol
    assert np.abs(var.double().cpu().numpy() - vref).max() <= ptol * np.abs(vref).max()
