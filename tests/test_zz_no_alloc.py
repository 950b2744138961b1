"""The product entry point that allocates nothing (glm_kernel_matmul_noalloc),
called through the C ABI: on two calls in a row, the second with a smaller
input, its result equals glm_kernel_matmul's bit for bit (same kernels, same
split plan) and lies within the rounding bound of the FP64 oracle:
  FP64 |got - ref| <= 1e-12 (K|V|);  FP32 <= 8 eps32 (8 + sqrt(n2)) (K|V|);
  BF16: relative l2 error <= 2e-3 (inputs rounded to BF16).
A product whose scratch exceeds the static maximum is refused with IGP_ENOMEM.
"""
import ctypes as ct
import math
import zlib

import numpy as np
import pytest
import torch

from oracle import kernels as ok
from paper_2310_20285_amd import _lib as L
from paper_2310_20285_amd import api

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)

# (n1, n2, d, C, nb): first call, then a smaller one on the same GPU
PAIRS = [
    ("fp32", "matern52", (3000, 3000, 16, 5, 1), (700, 1500, 16, 5, 1)),   # symmetric, then one-sided
    ("fp32", "rbf", (1200, 2311, 32, 5, 4), (1200, 1200, 32, 5, 1)),
    ("fp32", "matern12", (900, 1000, 7, 3, 2), (10, 33, 7, 3, 1)),        # direct-difference kernel
    ("fp64", "matern32", (800, 900, 4, 3, 1), (65, 77, 4, 3, 1)),
    ("bf16", "rbf", (1000, 1000, 100, 10, 1), (300, 513, 100, 10, 1)),
]


def _dev(a, dt):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _call(Xd1, Xd2, Vd, C, kind, ell, os_, prec):
    a = api.glm_kernel_matmul(Xd1, Xd2, Vd, C, kind, ell, os_, prec)
    out = torch.full_like(a, float("nan"))
    b = api.glm_kernel_matmul_noalloc(Xd1, Xd2, Vd, C, kind, ell, os_, prec, out=out)
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("case", PAIRS, ids=lambda c: f"{c[0]}-{c[1]}")
def test_noalloc_matches_workspace_entry(gpu_lib, case):
    prec, kind, first, second = case
    dt = torch.float64 if prec == "fp64" else torch.float32
    for shape in (first, second):
        n1, n2, d, C, nb = shape
        ell, os_ = 0.85 * math.sqrt(d), 0.8    # r / l of order one for N(0, I_d) rows
        print(f"noalloc {prec} {kind} shape={shape}", flush=True)
        rng = np.random.default_rng(zlib.crc32(repr((prec, kind, shape)).encode()))
        X2 = rng.standard_normal((n2, d))
        # X1 == X2 (same tensor) on square shapes, so the symmetric kernel runs
        same = n1 == n2
        X1 = X2 if same else rng.standard_normal((n1, d))
        V = rng.standard_normal((nb, n2 * C))
        Xd2 = _dev(X2, dt)
        Xd1 = Xd2 if same else _dev(X1, dt)
        Vd = _dev(V, dt)
        a, b = _call(Xd1, Xd2, Vd, C, kind, ell, os_, prec)
        assert torch.equal(a, b), f"{shape}: no-allocation result differs from glm_kernel_matmul"
        X1h, X2h, Vh = (t.double().cpu().numpy() for t in (Xd1, Xd2, Vd))
        K = ok.kernel_matrix(X1h, X2h, kind, ell, os_)
        got = b.double().cpu().numpy().reshape(nb, n1, C)
        for j in range(nb):
            Vj = Vh[j].reshape(n2, C)
            ref = K @ Vj
            if prec == "bf16":
                rel = np.linalg.norm(got[j] - ref) / np.linalg.norm(ref)
                assert rel <= 2e-3, f"{shape} vector {j}: relative error {rel:.2e}"
            else:
                tol = 1e-12 if prec == "fp64" else 8 * EPS32 * (8 + math.sqrt(n2))
                scale = K @ np.abs(Vj)
                err = np.abs(got[j] - ref)
                assert (err <= tol * scale + 1e-300).all(), \
                    f"{shape} vector {j}: max err/scale {(err / scale).max():.2e} > {tol:.2e}"


def test_noalloc_refuses_beyond_maximum(gpu_lib):
    lib = L.load()
    cap = lib.glm_kernel_matmul_noalloc_max_bytes()
    n, d, C = 30000, 16, 5
    need = lib.glm_kernel_matmul_ws_bytes(n, n, d, C, 1, L.IGP_FP32)
    assert need > cap
    X = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    V = torch.zeros(n * C, dtype=torch.float32, device="cuda")
    out = torch.full((n * C,), 3.0, dtype=torch.float32, device="cuda")
    kp, n_kp = api.kernel_params("matern52", 2.0, 1.0)
    code = lib.glm_kernel_matmul_noalloc(kp, n_kp, ct.c_void_p(X.data_ptr()), n,
                                         ct.c_void_p(X.data_ptr()), n, d,
                                         ct.c_void_p(V.data_ptr()), C, 1, n * C,
                                         ct.c_void_p(out.data_ptr()), n * C, 0.0, L.IGP_FP32,
                                         ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == L.IGP_ENOMEM
    assert b"no-allocation" in lib.igp_last_error()
    torch.cuda.synchronize()
    assert bool((out == 3.0).all()), "a refused call must not touch the output"
