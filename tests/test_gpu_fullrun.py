"""Free-running fits at the benchmark sizes against the FP64 O-method reference
(Algorithms 1-3 on the CPU, stored by tests/golden/make_fullsize_golden.py,
which calls only the oracle):

* N=20000, D=16, C=5, Matern-5/2, IterNCGP-CG j <= 200, R = 100, 5 Newton
  steps from f_0 = 0, FP32 products and FP64 projected solves, both residual
  modes.  Compared: the Newton iterates f_i (Algorithm 1) at 256 stored rows
  after every step, the log posterior Psi, and after the last step the
  predictive mean m_{i,j} at 256 test points.  Tolerance: 1e-4 relative
  (the stated target for the mean).
* image-shaped N=60000, D=784, C=10, RBF, CG j <= 5, R = inf, 3 Newton steps
  in each precision mode: FP32 and the split BF16 mode within 1e-4, plain
  BF16 at its measured level (about 4e-4; it does not meet the target).

The solver actions are the FP32 residuals, so iteration counts can differ by
a few from the FP64 run (both stop at the same tolerance); the comparison is
of the iterates, which both runs determine to that tolerance.  The marginal
variance depends on the span of the actions taken, not only on the solution,
so it is checked against the oracle's formula on the model's own root Q
(1e-4 of the prior variance) and its distance to the FP64 run is printed.
"""
import json
import os

import numpy as np
import pytest
import torch

import datagen
from oracle import predict as op
from paper_2310_20285_amd import api

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    with open(os.path.join(HERE, "golden", f"omethod_{name}.json")) as f:
        return json.load(f)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _var_own_root(m, w, Xt, var_gpu, X):
    """Max error of the model's variance against the oracle's formula on the
    model's own root Q and its FP32 inputs, relative to the prior variance."""
    Q = m.view(2).double().cpu().numpy().T          # (N*C, B)
    ref = op.predictive_var_root(Xt, X, Q, w.C, w.kernel, w.lengthscale, w.outputscale)
    return float(np.abs(var_gpu - ref).max() / w.outputscale)


@pytest.mark.parametrize("residual", ["recurrence", "explicit"])
def test_config2_free_running_fit_matches_fp64_omethod(gpu_lib, residual):
    g = _golden("config2")
    w = datagen.config2()
    assert (w.N, w.D, w.C, w.kernel) == (g["N"], g["D"], g["C"], g["kernel"])
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
    y = torch.tensor(w.y, dtype=torch.int32, device="cuda")
    m = api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="cg",
                     j_max=g["j_max"], rank_limit=g["rank_limit"], recycle=True,
                     tol_abs=1e-5, tol_rel=1e-5, precision="fp32", residual_mode=residual,
                     max_buffer=g["j_max"] + g["rank_limit"])
    rows = np.asarray(g["rows"])
    for i, ref in enumerate(g["steps"]):
        info = m.newton_step()
        F = m.view(0).double().cpu().numpy().reshape(w.N, w.C)
        e_f = _rel(F[rows], np.asarray(ref["F_rows"]))
        e_psi = abs(info["psi"] - ref["psi"]) / abs(ref["psi"])
        print(f"step {i + 1} ({residual}): iters {info['iters']} (FP64 {ref['iters']}), "
              f"F rel err {e_f:.2e}, psi rel err {e_psi:.2e}", flush=True)
        assert e_f <= 1e-4, f"step {i + 1}: Newton iterate off by {e_f:.2e}"
        assert e_psi <= 1e-6, f"step {i + 1}: psi off by {e_psi:.2e}"
        assert abs(info["iters"] - ref["iters"]) <= max(3, ref["iters"] // 5)
    Xs = torch.tensor(w.Xs[:g["test_points"]], dtype=torch.float32, device="cuda")
    mean, var, _ = m.predict(Xs)
    mean = mean.double().cpu().numpy()
    var = var.double().cpu().numpy()
    e_mean = _rel(mean, np.asarray(g["mean"]))
    e_var = _var_own_root(m, w, Xs.double().cpu().numpy(), var, X.double().cpu().numpy())
    d_var = float(np.abs(var - np.asarray(g["var"])).max() / w.outputscale)
    print(f"predictive mean rel err {e_mean:.2e}; variance vs own-root oracle {e_var:.2e}, "
          f"vs the FP64 run {d_var:.2e}", flush=True)
    assert e_mean <= 1e-4
    assert e_var <= 1e-4


# image-shaped N=60000, D=784, C=10, RBF, CG j <= 5, R = inf, 3 Newton steps.
# FP32 products run the direct-difference kernel (D > 128).  Plain BF16 is
# asserted at its measured level (4.2e-4 on the iterates, 3.6e-4 on the mean).
IMAGE_TOL = {"fp32": 1e-4, "bf16x3": 1e-4, "bf16": 6e-4}


@pytest.mark.parametrize("prec", ["bf16", "bf16x3", "fp32"])
def test_image_fit_matches_fp64_omethod(gpu_lib, prec):
    g = _golden("config3")
    w = datagen.config3(Ns=1000)
    assert (w.N, w.D, w.C, w.kernel) == (g["N"], g["D"], g["C"], g["kernel"])
    assert abs(w.lengthscale - g["lengthscale"]) <= 1e-12 * g["lengthscale"]
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
    y = torch.tensor(w.y, dtype=torch.int32, device="cuda")
    m = api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="cg",
                     j_max=g["j_max"], rank_limit=-1, recycle=True, tol_abs=1e-5, tol_rel=1e-5,
                     precision=prec, residual_mode="recurrence",
                     max_buffer=g["j_max"] * len(g["steps"]) + 1)
    rows = np.asarray(g["rows"])
    errs = []
    for i, ref in enumerate(g["steps"]):
        info = m.newton_step()
        F = m.view(0).double().cpu().numpy().reshape(w.N, w.C)
        e_f = _rel(F[rows], np.asarray(ref["F_rows"]))
        errs.append(e_f)
        print(f"{prec} step {i + 1}: iters {info['iters']} (FP64 {ref['iters']}), "
              f"F rel err {e_f:.2e}, psi {info['psi']:.6f} (FP64 {ref['psi']:.6f})", flush=True)
        assert info["iters"] == ref["iters"]
    Xs = torch.tensor(w.Xs[:g["test_points"]], dtype=torch.float32, device="cuda")
    mean, var, _ = m.predict(Xs)
    var = var.double().cpu().numpy()
    e_mean = _rel(mean.double().cpu().numpy(), np.asarray(g["mean"]))
    e_var = _var_own_root(m, w, Xs.double().cpu().numpy(), var, X.double().cpu().numpy())
    d_var = float(np.abs(var - np.asarray(g["var"])).max())
    print(f"{prec}: predictive mean rel err {e_mean:.2e}; variance vs own-root oracle "
          f"{e_var:.2e}, vs the FP64 run {d_var:.2e}", flush=True)
    assert max(errs) <= IMAGE_TOL[prec]
    assert e_mean <= IMAGE_TOL[prec]
    assert e_var <= max(IMAGE_TOL[prec], 1e-4)
