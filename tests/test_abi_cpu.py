"""Host-side checks of the C ABI: the library loads without a GPU, exports
every function include/itergp.h declares, and its host-only entry points
(size queries, argument checks, the FP64 eigensolver) behave."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2310_20285_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "itergp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ("glm_kernel_matmul", "glm_softmax_hessian_apply", "itergp_newton_step",
                 "itergp_predict", "itergp_init", "itergp_state_bytes"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    lib = L.load()
    missing = [f for f in header_functions() if not hasattr(lib, f)]
    assert not missing, missing
    assert set(L.SIGNATURES) >= set(header_functions())


def test_version_and_error_string():
    lib = L.load()
    assert lib.igp_version().startswith(b"itergp")
    assert lib.igp_last_error() is not None


def test_state_bytes_queries():
    lib = L.load()
    cfg = L.SolverConfig(0, 200, 100, 1, 1e-5, 1e-5, L.IGP_FP32, 0, 300, 0)
    b = lib.itergp_state_bytes(20000, 16, 5, ct.byref(cfg))
    # dominated by five N*C x B buffers (S, T, Q and two re-weighting targets)
    assert 5 * 20000 * 5 * 300 * 4 <= b <= 8 * 20000 * 5 * 300 * 4
    cfg2 = L.SolverConfig(0, 200, 100, 1, 1e-5, 1e-5, L.IGP_FP32, 0, 600, 0)
    assert lib.itergp_state_bytes(20000, 16, 5, ct.byref(cfg2)) > b
    cfg0 = L.SolverConfig(0, 200, 100, 1, 1e-5, 1e-5, L.IGP_FP32, 0, 0, 0)
    assert lib.itergp_state_bytes(20000, 16, 5, ct.byref(cfg0)) == 0
    assert lib.glm_kernel_matmul_ws_bytes(1000, 1000, 16, 5, 1, L.IGP_FP32) > 0
    assert lib.glm_kernel_matmul_ws_bytes(-1, 1000, 16, 5, 1, L.IGP_FP32) == 0


def test_argument_errors_without_device_work():
    lib = L.load()
    kp = L.KernelParams(L.IGP_RBF, 0, -1.0, 1.0)
    rc = lib.glm_kernel_matmul(ct.byref(kp), 1, None, 4, None, 4, 2, None, 1, 1, 4, None, 4, 0.0,
                               L.IGP_FP32, None, 0, None)
    assert rc == L.IGP_EINVAL
    assert b"hyperparameters" in lib.igp_last_error()
    kp = L.KernelParams(7, 0, 1.0, 1.0)
    assert lib.glm_kernel_matmul(ct.byref(kp), 1, None, 4, None, 4, 2, None, 1, 1, 4, None, 4, 0.0,
                                 L.IGP_FP32, None, 0, None) == L.IGP_EINVAL
    kp = L.KernelParams(L.IGP_RBF, 0, 1.0, 1.0)
    # empty problems are no-ops that touch nothing
    assert lib.glm_kernel_matmul(ct.byref(kp), 1, None, 0, None, 4, 2, None, 1, 1, 4, None, 4, 0.0,
                                 L.IGP_FP32, None, 0, None) == L.IGP_OK
    assert lib.glm_softmax_hessian_apply(None, 0, 3, None, 1, 0, None, 0, L.IGP_W_PINV,
                                         L.IGP_FP32, None) == L.IGP_OK
    assert lib.glm_softmax_hessian_apply(None, 4, 3, None, 1, 12, None, 12, 5, L.IGP_FP32,
                                         None) == L.IGP_EINVAL
    # one kernel per class: n_kp must be 1 or C, one kernel family
    kp3 = (L.KernelParams * 3)(L.KernelParams(L.IGP_RBF, 0, 1.0, 1.0),
                               L.KernelParams(L.IGP_RBF, 0, 2.0, 1.0),
                               L.KernelParams(L.IGP_MATERN32, 0, 1.0, 1.0))
    assert lib.glm_kernel_matmul(kp3, 2, None, 4, None, 4, 2, None, 3, 1, 12, None, 12, 0.0,
                                 L.IGP_FP32, None, 0, None) == L.IGP_EINVAL
    assert b"n_kp" in lib.igp_last_error()
    assert lib.glm_kernel_matmul(kp3, 3, None, 4, None, 4, 2, None, 3, 1, 12, None, 12, 0.0,
                                 L.IGP_FP32, None, 0, None) == L.IGP_EINVAL
    assert b"family" in lib.igp_last_error()
    h = ct.c_void_p()
    cfg = L.SolverConfig(0, 10, -1, 1, 1e-5, 1e-5, L.IGP_FP32, 0, 5, 0)   # max_buffer < j_max
    assert lib.itergp_init(ct.byref(h), ct.byref(kp), 1, ct.byref(cfg), ct.c_void_p(1),
                           ct.c_void_p(1), 10, 2, 3, ct.c_void_p(256), 1 << 30,
                           None) == L.IGP_EINVAL
    assert b"max_buffer" in lib.igp_last_error()
    for lik, noise, msg in ((7, 1.0, b"likelihood"), (L.IGP_LIK_GAUSSIAN, 0.0, b"noise_var"),
                            (L.IGP_LIK_GAUSSIAN, float("nan"), b"noise_var")):
        cfg = L.SolverConfig(0, 10, -1, 1, 1e-5, 1e-5, L.IGP_FP32, 0, 20, lik, noise)
        assert lib.itergp_init(ct.byref(h), ct.byref(kp), 1, ct.byref(cfg), ct.c_void_p(1),
                               ct.c_void_p(1), 10, 2, 1, ct.c_void_p(256), 1 << 30,
                               None) == L.IGP_EINVAL
        assert msg in lib.igp_last_error()


def test_batched_step_argument_errors_without_device_work():
    """The batched step refuses unknown flags and an empty batch before it
    touches a model or the device."""
    lib = L.load()
    rc = lib.itergp_newton_step_batched_ex(None, 1, None, None, 0,
                                           L.IGP_BATCH_DEVICE_CONTROL << 1)
    assert rc == L.IGP_EINVAL
    assert b"flags" in lib.igp_last_error()
    assert lib.itergp_newton_step_batched_ex(None, 0, None, None, 0,
                                             L.IGP_BATCH_DEVICE_CONTROL) == L.IGP_EINVAL
    assert b"no models" in lib.igp_last_error()
    assert lib.itergp_newton_step_batched(None, 0, None, None, 0) == L.IGP_EINVAL


@pytest.mark.parametrize("n", [1, 2, 7, 40, 150])
def test_host_eigh_matches_numpy(n):
    lib = L.load()
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n))
    A = G @ G.T + np.diag(np.linspace(0, 1, n))
    w = np.empty(n)
    Z = np.empty((n, n))         # row k = eigenvector k (column-major Z)
    rc = lib.igp_host_eigh(n, A.ctypes.data, w.ctypes.data, Z.ctypes.data)
    assert rc == L.IGP_OK
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    np.testing.assert_allclose(w, ref, rtol=1e-11, atol=1e-11 * ref[0])
    U = Z.T
    np.testing.assert_allclose(U.T @ U, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(U @ np.diag(w) @ U.T, A, atol=1e-11 * np.abs(A).max())


def test_host_eigh_degenerate_spectrum():
    lib = L.load()
    n = 30
    rng = np.random.default_rng(0)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([3.0, 1.0, 0.0], 10)
    A = (Qm * lam) @ Qm.T
    w, Z = np.empty(n), np.empty((n, n))
    assert lib.igp_host_eigh(n, A.ctypes.data, w.ctypes.data, Z.ctypes.data) == 0
    np.testing.assert_allclose(w, lam, atol=1e-12)
    U = Z.T
    np.testing.assert_allclose(U @ np.diag(w) @ U.T, A, atol=1e-12)


def test_batched_tuning_table_round_trip():
    """The launch-shape table loads from the JSON itergp_batched_tuning
    writes (FP32 and BF16 entries are separate keys), keeps entries it already
    has, and refuses malformed or out-of-range entries (host only, no device
    work)."""
    import json

    from paper_2310_20285_amd import api
    entries = [{"precision": "fp32", "kind": 2, "feature_chunks": 1, "log2_rows": 13,
                "strips": 2, "split_rows": 1024, "us": 812.5},
               {"kind": 3, "feature_chunks": 2, "log2_rows": 17, "strips": 1,
                "split_rows": 4096}]
    added = api.batched_tuning_load(json.dumps(entries))
    assert added == 2
    table = json.loads(api.batched_tuning())
    keys = {(e["precision"], e["kind"], e["feature_chunks"], e["log2_rows"]):
            (e["strips"], e["split_rows"]) for e in table}
    assert keys[("fp32", 2, 1, 13)] == (2, 1024) and keys[("fp32", 3, 2, 17)] == (1, 4096)
    # a BF16 entry of the same shape is a different key
    bf = dict(entries[0], precision="bf16", strips=1)
    assert api.batched_tuning_load(json.dumps([bf])) == 1
    keys = {(e["precision"], e["kind"], e["feature_chunks"], e["log2_rows"]):
            (e["strips"], e["split_rows"]) for e in json.loads(api.batched_tuning())}
    assert keys[("bf16", 2, 1, 13)] == (1, 1024) and keys[("fp32", 2, 1, 13)] == (2, 1024)
    # the same entries again add nothing; a different value for a known key
    # does not replace it
    assert api.batched_tuning_load(json.dumps(entries)) == 0
    other = dict(entries[1], strips=2)
    assert api.batched_tuning_load(json.dumps([other])) == 0
    table = json.loads(api.batched_tuning())
    assert [e["strips"] for e in table if (e["kind"], e["log2_rows"]) == (3, 17)] == [1]
    for bad in ('[{"kind": 2, "feature_chunks": 1, "log2_rows": 13, "strips": 3, '
                '"split_rows": 1024}]',
                '[{"kind": 2, "feature_chunks": 1, "log2_rows": 13, "strips": 1}]',
                '[{"precision": "fp64", "kind": 2, "feature_chunks": 1, "log2_rows": 13, '
                '"strips": 1, "split_rows": 1024}]',
                '[{"kind": 2, "feature_chunks": 1'):
        with pytest.raises(L.IterGPError) as e:
            api.batched_tuning_load(bad)
        assert e.value.code == L.IGP_EINVAL
