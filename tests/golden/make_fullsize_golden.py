"""Write the FP64 O-method reference of the two benchmark-size fits.

    python tests/golden/make_fullsize_golden.py config2   # N=20000: ~10 min, ~8 GB RAM
    python tests/golden/make_fullsize_golden.py config3   # N=60000: ~15 min, ~36 GB RAM
    python tests/golden/make_fullsize_golden.py products  # sampled rows of single products

Calls only ``oracle/`` (the FP64 CPU reference) and ``datagen/`` (the seeded
inputs).  The inputs are the arrays the GPU receives: X and the test points
rounded to FP32 (then held in FP64 here).  The kernel matrix K_X is formed
once in FP64 and kept in memory; every product with K in Algorithms 1-3 is
then K_X times a CN-ordered vector.

config2: X ~ N(0, I_16), N = 20000, C = 5, Matern-5/2 (l = 2, os = 1);
         IterNCGP with residual (CG) actions, j <= 200 per Newton step,
         compression to R = 100 at every virtual solver run, 5 Newton steps
         from f_0 = 0 (outer stop off).
config3: image-shaped N = 60000, D = 784, C = 10, RBF (median lengthscale);
         CG actions, j <= 5, R = infinity, 3 Newton steps.

products: one product K(X, X) v at each benchmark size (the N=20000 and the
         image-shaped N=60000 inputs), v ~ N(0, 1) seeded and rounded to FP32,
         FP64 values at 64 seeded rows (the last row included).

Stored (JSON): per Newton step the iteration count, the last residual norm,
the number of recycled columns, ||F||, the relative change and Psi; F at 256
seeded rows after every step; the predictive mean and marginal variance
(eqs. for m_{i,j} and k_{i,j}) at the first 256 test points after the last
step.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import datagen                                   # noqa: E402
from oracle import itergp as oi                  # noqa: E402
from oracle import kernels as ok                 # noqa: E402
from oracle import newton as on                  # noqa: E402
from oracle import predict as op                 # noqa: E402

N_ROWS = 256
N_TEST = 256

CONFIGS = {
    "config2": dict(make=lambda: datagen.config2(), steps=5, j_max=200, rank_limit=100,
                    gram=False,
                    workload="gpc N=20000 D=16 C=5 matern52 l=2 os=1, seed 1; "
                             "IterNCGP-CG j<=200 R=100, 5 Newton steps from f_0=0"),
    "config3": dict(make=lambda: datagen.config3(Ns=1000), steps=3, j_max=5, rank_limit=-1,
                    gram=True,
                    workload="image-shaped N=60000 D=784 C=10 rbf (median lengthscale), seed 2; "
                             "IterNCGP-CG j<=5 R=inf, 3 Newton steps from f_0=0"),
}


def as_fp32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def run(name: str) -> str:
    cfg = CONFIGS[name]
    t0 = time.time()
    w = cfg["make"]()
    X, Xs = as_fp32(w.X), as_fp32(w.Xs)
    N, C = w.N, w.C
    print(f"{name}: N={N} D={w.D} C={C} {w.kernel} l={w.lengthscale:.6g}", flush=True)
    if cfg["gram"]:
        KX = ok.kernel_matrix_gram(X, X, w.kernel, w.lengthscale, w.outputscale)
    else:
        KX = ok.kernel_matrix(X, X, w.kernel, w.lengthscale, w.outputscale)
    print(f"  K formed ({time.time() - t0:.0f} s)", flush=True)
    count = [0]

    def apply_K(V):
        count[0] += 1
        return ok.apply_full_kernel_cn(KX, V, C)

    recs = oi.iterncgp(apply_K, w.y, C, cfg["steps"], policy="cg", j_max=cfg["j_max"],
                       rank_limit=cfg["rank_limit"], recycle=True)
    print(f"  {len(recs)} Newton steps, {count[0]} products ({time.time() - t0:.0f} s)",
          flush=True)
    rows = np.sort(np.random.default_rng(12345).choice(N, size=N_ROWS, replace=False))
    Xt = Xs[:N_TEST]
    mean = op.predictive_mean(Xt, X, recs[-1].v, C, w.kernel, w.lengthscale, w.outputscale)
    var = op.predictive_var_root(Xt, X, recs[-1].Q, C, w.kernel, w.lengthscale, w.outputscale)
    steps = []
    for rec in recs:
        steps.append({
            "iters": rec.info.iters,
            "converged": bool(rec.info.converged),
            "res_norm_last": rec.info.res_norms[-1] if rec.info.res_norms else None,
            "rhs_norm": rec.info.rhs_norm,
            "recycled_cols": int(rec.info.vsr.eigvals.size) if rec.info.vsr else 0,
            "F_norm": float(np.linalg.norm(rec.F)),
            "rel_change": rec.rel_change,
            "psi": on.psi_from_v(rec.F, w.y, rec.v),
            "F_rows": rec.F[rows].tolist(),
        })
    out = {
        "workload": cfg["workload"],
        "inputs": "datagen seeded workload; X and test points rounded to FP32",
        "N": N, "D": w.D, "C": C, "kernel": w.kernel, "lengthscale": w.lengthscale,
        "outputscale": w.outputscale, "j_max": cfg["j_max"], "rank_limit": cfg["rank_limit"],
        "rows": rows.tolist(), "test_points": N_TEST,
        "steps": steps,
        "mean": mean.tolist(), "var": var.tolist(),
        "products": count[0], "seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(HERE, f"omethod_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"  wrote {path} ({time.time() - t0:.0f} s)", flush=True)
    return path


def run_products() -> str:
    out = {}
    for name, make, gram in (("config2", lambda: datagen.config2(), False),
                             ("config3", lambda: datagen.config3(Ns=1000), True)):
        w = make()
        X = as_fp32(w.X)
        rng = np.random.default_rng(2024)
        v = as_fp32(rng.standard_normal(w.N * w.C))
        rows = np.sort(rng.choice(w.N, size=64, replace=False))
        rows[-1] = w.N - 1
        kmat = ok.kernel_matrix_gram if gram else ok.kernel_matrix
        K = kmat(X[rows], X, w.kernel, w.lengthscale, w.outputscale)
        ref = K @ v.reshape(w.N, w.C)
        out[name] = {"N": w.N, "D": w.D, "C": w.C, "kernel": w.kernel,
                     "lengthscale": w.lengthscale, "outputscale": w.outputscale,
                     "v": "numpy default_rng(2024).standard_normal(N*C) rounded to FP32; "
                          "rows drawn next from the same generator (64, last row forced)",
                     "rows": rows.tolist(), "ref": ref.tolist()}
        print(f"products {name}: done", flush=True)
    path = os.path.join(HERE, "kv_products.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    return path


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["config2"]:
        run_products() if nm == "products" else run(nm)
