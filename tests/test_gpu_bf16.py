"""GPU checks of the BF16 precision modes (distance GEMM on BF16 MFMA with FP32
accumulation, inputs rounded to BF16 after centring, norms of the rounded
rows; contraction with V as BF16 hi/lo parts).  "bf16x3" splits each input
into BF16 high and low parts and takes three products (hh + lh + hl).

Tolerance of one product (first order, per output entry n, c):

  |got - ref| <= sum_m  Lk/l^2 * dr2_nm * |V[m, c]|  +  tol32 * (K|V|)[n, c]

  dr2_nm = 2u sum_d |a_d - b_d| (|a_d| + |b_d|) + (2u^2 + e_ll) (|a|^2 + |b|^2)
           + 4 sqrt(P D) eps32 (|a|^2 + |b|^2)        (rounding a, b to BF16 with
                                                        unit roundoff u = 2^-8, and the
                                                        FP32 norm expansion over P D
                                                        products)
  bf16: u = 2^-8, e_ll = 0, P = 1;  bf16x3: the represented input h + l is
  within 2^-8 |x - h| <= 2^-16 |x| of x (u = 2^-16), the dropped l.l term adds
  e_ll = 2^-16, P = 3.
  Lk = max |dk/d(r^2/l^2)| / os: 1/2 (RBF), 3/2 (Matern-3/2), 5/6 (Matern-5/2)
  tol32 = 8 eps32 (8 + sqrt(n2)) + 2^-15               (FP32 sums, BF16 hi/lo products)

with a, b the centred rows and ref the FP64 oracle on the unrounded inputs.
"""
import math

import numpy as np
import pytest
import torch

import datagen
from oracle import itergp as oi
from oracle import kernels as ok
from oracle import predict as op
from paper_2310_20285_amd import api

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)
U_BF16 = 2.0 ** -8
LK = {"rbf": 0.5, "matern32": 1.5, "matern52": 5.0 / 6.0}


MODE = {"bf16": (U_BF16, 0.0, 1), "bf16x3": (2.0 ** -16, 2.0 ** -16, 3)}


def _bound(X1, X2, V, C, kind, ell, os_, mode="bf16"):
    u, e_ll, nprod = MODE[mode]
    c = X2.mean(axis=0)
    A, B = X1 - c, X2 - c
    D = A.shape[1]
    na, nb = (A * A).sum(1), (B * B).sum(1)
    absd = np.zeros((A.shape[0], B.shape[0]))
    for d in range(D):
        absd += np.abs(A[:, d, None] - B[None, :, d]) * (np.abs(A[:, d, None]) + np.abs(B[None, :, d]))
    dr2 = (2 * u * absd + (2 * u ** 2 + e_ll + 4 * math.sqrt(nprod * D) * EPS32)
           * (na[:, None] + nb[None, :]))
    K = ok.kernel_matrix(X1, X2, kind, ell, os_)
    n2 = X2.shape[0]
    tol32 = 8 * EPS32 * (8 + math.sqrt(n2)) + 2.0 ** -15
    Va = np.abs(V).reshape(n2, C)
    return (os_ * LK[kind] / ell ** 2) * (dr2 @ Va) + tol32 * (K @ Va), K


@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
@pytest.mark.parametrize("kind", ["rbf", "matern32", "matern52"])
@pytest.mark.parametrize("shape", [(200, 300, 784, 10), (130, 257, 40, 3), (64, 129, 8, 1),
                                   (257, 520, 100, 16)])
def test_bf16_kernel_matmul_within_rounding_bound(gpu_lib, kind, shape, mode):
    n1, n2, d, C = shape
    rng = np.random.default_rng(n1 + n2 + d)
    X1 = rng.uniform(0.0, 1.0, size=(n1, d)) * (rng.uniform(size=(n1, d)) < 0.3)
    X2 = rng.uniform(0.0, 1.0, size=(n2, d)) * (rng.uniform(size=(n2, d)) < 0.3)
    V = rng.standard_normal(n2 * C)
    ell = math.sqrt(0.3 * d)
    Xd1 = torch.tensor(X1, dtype=torch.float32, device="cuda")
    Xd2 = torch.tensor(X2, dtype=torch.float32, device="cuda")
    Vd = torch.tensor(V, dtype=torch.float32, device="cuda")
    X1h, X2h, Vh = (t.double().cpu().numpy() for t in (Xd1, Xd2, Vd))
    out = api.glm_kernel_matmul(Xd1, Xd2, Vd, C, kind, ell, 0.8, mode).double().cpu().numpy()
    bound, K = _bound(X1h, X2h, Vh, C, kind, ell, 0.8, mode)
    ref = (K @ Vh.reshape(n2, C)).reshape(-1)
    err = np.abs(out - ref)
    assert np.all(err <= 2.0 * bound.reshape(-1)), (err / bound.reshape(-1)).max()


@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
@pytest.mark.parametrize("kind", ["rbf", "matern52"])
@pytest.mark.parametrize("shape", [(1, 8, 2), (300, 784, 10), (513, 40, 3), (257, 100, 16),
                                   (300, 20, 17)])
def test_bf16_symmetric_within_rounding_bound(gpu_lib, kind, shape, mode):
    """Same rows on both sides: each pair of 256-row blocks evaluated once (a
    ragged last block, up to W = 16 output columns; W = 17 takes the one-sided
    kernel), same bound as the one-sided product."""
    n, d, C = shape
    rng = np.random.default_rng(n + d + C)
    X = rng.uniform(0.0, 1.0, size=(n, d)) * (rng.uniform(size=(n, d)) < 0.3)
    V = rng.standard_normal(n * C)
    ell = math.sqrt(0.3 * d)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Vd = torch.tensor(V, dtype=torch.float32, device="cuda")
    Xh, Vh = (t.double().cpu().numpy() for t in (Xd, Vd))
    out = api.glm_kernel_matmul(Xd, Xd, Vd, C, kind, ell, 0.8, mode).double().cpu().numpy()
    bound, K = _bound(Xh, Xh, Vh, C, kind, ell, 0.8, mode)
    ref = (K @ Vh.reshape(n, C)).reshape(-1)
    err = np.abs(out - ref)
    assert np.all(err <= 2.0 * bound.reshape(-1)), (err / bound.reshape(-1)).max()


@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
def test_bf16_symmetric_matches_one_sided(gpu_lib, mode):
    rng = np.random.default_rng(5)
    X = torch.tensor(rng.uniform(0.0, 1.0, size=(2600, 784)), dtype=torch.float32, device="cuda")
    V = torch.tensor(rng.standard_normal((2, 2600 * 10)), dtype=torch.float32, device="cuda")
    sym = api.glm_kernel_matmul(X, X, V, 10, "rbf", 12.0, 1.0, mode)
    one = api.glm_kernel_matmul(X, X.clone(), V, 10, "rbf", 12.0, 1.0, mode)
    assert ((sym - one).norm() / one.norm()).item() <= 1e-5
    again = api.glm_kernel_matmul(X, X, V, 10, "rbf", 12.0, 1.0, mode)
    assert torch.equal(sym, again)


# error against FP64 with the oracle's actions replayed: the split mode meets
# the 1e-4 target; plain BF16 does not (measured on this problem: iterates up
# to 1.3e-3, predictive mean 4.6e-4; asserted at 2e-3)
MODEL_TOL = {"bf16": 2e-3, "bf16x3": 1e-4}


@pytest.mark.parametrize("mode", ["bf16", "bf16x3"])
def test_bf16_model_error_vs_fp64_oracle(gpu_lib, mode):
    """IterNCGP on an image-shaped problem in a BF16 mode with the oracle's
    actions replayed: Newton iterates and predictive mean against FP64."""
    w = datagen.image_like(seed=12, N=900, Ns=200)
    n = w.N * w.C
    KX = ok.kernel_matrix(w.X, w.X, w.kernel, w.lengthscale, w.outputscale)
    recs = oi.iterncgp(lambda V: ok.apply_full_kernel_cn(KX, V, w.C), w.y, w.C, 3, policy="cg",
                       j_max=5, rank_limit=-1, recycle=True)
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
    y = torch.tensor(w.y, dtype=torch.int32, device="cuda")
    m = api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="user", j_max=5,
                     rank_limit=-1, recycle=True, precision=mode, max_buffer=15)
    errs = []
    for rec in recs:
        m.set_user_actions(torch.tensor(np.stack(rec.info.actions), dtype=torch.float32,
                                        device="cuda"))
        m.newton_step()
        F = m.view(0).double().cpu().numpy().reshape(w.N, w.C)
        errs.append(np.linalg.norm(F - rec.F) / np.linalg.norm(rec.F))
    Xs = torch.tensor(w.Xs, dtype=torch.float32, device="cuda")
    mean, var, _ = m.predict(Xs, probs=False)
    mref = op.predictive_mean(w.Xs, w.X, recs[-1].v, w.C, w.kernel, w.lengthscale,
                              w.outputscale)
    em = np.linalg.norm(mean.double().cpu().numpy() - mref) / np.linalg.norm(mref)
    print(f"{mode} vs FP64: Newton iterates rel err {errs}, predictive mean rel err {em:.2e}")
    assert max(errs) <= MODEL_TOL[mode] and em <= MODEL_TOL[mode]
