"""GPU parity of the two standalone boundary calls against the FP64 oracle:
glm_kernel_matmul and glm_softmax_hessian_apply.

Tolerances (rounding bounds of each precision):
  FP64: |got - ref| <= 1e-12 * (K |V|)            (rounding of ~n2 FP64 terms)
  FP32: |got - ref| <= 8 eps32 (8 + sqrt(n2)) * (K |V|)
where K |V| is the oracle product with |V|, the natural scale of each entry.
"""
import math
import zlib

import numpy as np
import pytest
import torch

from datagen import KERNEL_KINDS
from oracle import kernels as ok
from oracle import likelihood as lk
from paper_2310_20285_amd import api

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


def _dev(a, dt):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _tol(prec, n2):
    return 1e-12 if prec == "fp64" else 8 * EPS32 * (8 + math.sqrt(max(n2, 1)))


SHAPES = [  # n1, n2, d, C, nb  -- several tiles plus ragged tails
    (200, 173, 3, 3, 1),
    (67, 300, 16, 5, 2),
    (130, 129, 33, 1, 3),
    (1, 1, 1, 1, 1),
    (257, 64, 8, 2, 1),
    (1000, 2311, 16, 5, 1),     # solver product shape (matrix-core path in FP32)
    (129, 700, 32, 5, 40),      # predict shape: W = C * nb = 200 output columns
    (70, 90, 128, 3, 2),        # widest feature count of the FP32 matrix-core path
    (150, 333, 3, 10, 1),       # at most 4 features, wide outputs (one-MFMA distance)
    (90, 260, 4, 5, 4),         # ... 20 output columns
    (70, 200, 1, 3, 17),        # ... 51 output columns
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", KERNEL_KINDS)
@pytest.mark.parametrize("shape", SHAPES)
def test_kernel_matmul_parity(gpu_lib, prec, kind, shape):
    n1, n2, d, C, nb = shape
    rng = np.random.default_rng(zlib.crc32(repr((prec, kind, shape)).encode()))
    X1 = rng.standard_normal((n1, d))
    X2 = rng.standard_normal((n2, d))
    V = rng.standard_normal((nb, n2 * C))
    ell, os_ = 1.3, 0.7
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xd1, Xd2, Vd = _dev(X1, dt), _dev(X2, dt), _dev(V, dt)
    # compare against the oracle on the values the device actually holds
    X1h, X2h, Vh = (t.double().cpu().numpy() for t in (Xd1, Xd2, Vd))
    out = api.glm_kernel_matmul(Xd1, Xd2, Vd, C, kind, ell, os_, prec).double().cpu().numpy()
    K = ok.kernel_matrix(X1h, X2h, kind, ell, os_)
    for b in range(nb):
        ref = (K @ Vh[b].reshape(n2, C)).reshape(-1)
        scale = (K @ np.abs(Vh[b]).reshape(n2, C)).reshape(-1)
        err = np.abs(out[b] - ref)
        assert np.all(err <= _tol(prec, n2) * scale + 1e-300), (err / scale).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_kernel_matmul_beta_and_empty(gpu_lib, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(5)
    X1, X2 = rng.standard_normal((50, 4)), rng.standard_normal((70, 4))
    V = rng.standard_normal(70 * 2)
    O0 = rng.standard_normal(50 * 2)
    Xd1, Xd2, Vd = _dev(X1, dt), _dev(X2, dt), _dev(V, dt)
    out = _dev(O0, dt)
    api.glm_kernel_matmul(Xd1, Xd2, Vd, 2, "rbf", 1.0, 1.0, prec, beta=0.5, out=out)
    ref = ok.kernel_matvec(Xd1.double().cpu().numpy(), Xd2.double().cpu().numpy(),
                           Vd.double().cpu().numpy().reshape(70, 2), "rbf", 1.0, 1.0).reshape(-1)
    ref = ref + 0.5 * out.new_tensor(O0).double().cpu().numpy()
    np.testing.assert_allclose(out.double().cpu().numpy(), ref, rtol=1e-5 if prec == "fp32" else 1e-12,
                               atol=1e-5 if prec == "fp32" else 1e-12)
    # n2 == 0: Out = beta * Out
    out2 = _dev(O0, dt)
    api.glm_kernel_matmul(Xd1, Xd2[:0], Vd[:0], 2, "rbf", 1.0, 1.0, prec, beta=2.0, out=out2)
    np.testing.assert_allclose(out2.double().cpu().numpy(), 2.0 * _dev(O0, dt).double().cpu().numpy(),
                               rtol=1e-15)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_kernel_matmul_deterministic(gpu_lib, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(6)
    X = _dev(rng.standard_normal((3000, 16)), dt)
    V = _dev(rng.standard_normal(3000 * 5), dt)
    a = api.glm_kernel_matmul(X, X, V, 5, "matern52", 2.0, 1.0, prec)
    b = api.glm_kernel_matmul(X, X, V, 5, "matern52", 2.0, 1.0, prec)
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("C", [1, 2, 3, 5, 10, 17])
@pytest.mark.parametrize("mode", ["w", "pinv"])
def test_softmax_hessian_apply_parity(gpu_lib, prec, C, mode):
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(C)
    N, nb = 333, 3
    F = rng.standard_normal((N, C)) * 2.0
    V = rng.standard_normal((nb, N * C))
    Fd, Vd = _dev(F, dt), _dev(V, dt)
    out = api.glm_softmax_hessian_apply(Fd, Vd, mode).double().cpu().numpy()
    Fh, Vh = Fd.double().cpu().numpy(), Vd.double().cpu().numpy()
    B = lk.softmax_hessian_pinv_blocks(Fh) if mode == "pinv" else lk.softmax_hessian_blocks(Fh)
    P = lk.softmax(Fh)
    tol = 1e-13 if prec == "fp64" else 64 * EPS32
    for b in range(nb):
        ref = lk.apply_blocks(B, Vh[b])
        a = np.abs(Vh[b]).reshape(N, C)
        # magnitude of the intermediates the block product forms (the rounding scale):
        # W v = pi*v - pi (pi^T v);  W^+ v = u/pi - mean(u/pi) with u = v - mean(v)
        if mode == "w":
            scale = P * a + P * (P * a).sum(1, keepdims=True)
        else:
            q = (a + a.mean(1, keepdims=True)) / P
            scale = q + q.mean(1, keepdims=True)
        scale = scale.reshape(-1) + 1e-30
        assert np.all(np.abs(out[b] - ref) <= tol * scale), (np.abs(out[b] - ref) / scale).max()
