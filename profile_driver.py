"""Profiling driver for rocprofv3.

    python profile_driver.py [--workload gpc16|image|predict|batched|gmm] [--precision ...]
                             [--reps 20] [--copy-mib 256]

Workloads (each ends with one device-to-device copy of ``--copy-mib`` MiB, a
transfer of known size whose FETCH_SIZE / WRITE_SIZE readings give the factor
that converts the counters of the other kernels to bytes):

* gpc16   the fused K.v product of the N=20000, D=16, C=5 Matern-5/2 workload
          in FP32 (the product each solver iteration issues), ``--reps`` times
          via glm_kernel_matmul;
* image   the fused K.v product of the image-shaped N=60000, D=784, C=10 RBF
          workload with the BF16 distance GEMM (``--precision bf16x3``: the
          split-input mode), ``--reps`` times;
* predict prediction (mean, variance, probit) at 4096 test points against a
          fitted N=100000, D=32, C=10 RBF model compressed to 100 directions
          (the serving workload's model), ``--reps`` times;
* batched 64 independent problems (N ~ U{1000..16000}, D=8, C ~ U{2..8},
          Matern-3/2, IterNCGP-CG j<=200, R=100) advanced by min(--reps, 3)
          batched Newton steps from f_0 = 0, launch shapes from the saved table
          (FP32, or ``--precision bf16``);
* gmm     the fused K.v product of the Gaussian-mixture workload (N=100000,
          D=3, C=10, Matern-3/2, lengthscale 0.05) in FP32, ``--reps`` times.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="gpc16",
                    choices=["gpc16", "image", "predict", "batched", "gmm"])
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16", "bf16x3"])
    args = ap.parse_args()

    import numpy as np
    import torch

    import datagen
    from paper_2310_20285_amd import api

    if args.workload in ("gpc16", "image", "gmm"):
        w = {"gpc16": datagen.config2, "image": lambda: datagen.config3(Ns=1000),
             "gmm": datagen.gmm}[args.workload]()
        prec = args.precision or ("bf16" if args.workload == "image" else "fp32")
        X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
        v = torch.randn(w.N * w.C, dtype=torch.float32, device="cuda")
        out = None
        for _ in range(args.reps):
            out = api.glm_kernel_matmul(X, X, v, w.C, w.kernel, w.lengthscale, w.outputscale,
                                        prec, out=out)
        what = f"{args.reps} K.v products (N={w.N}, D={w.D}, C={w.C}, {prec})"
    elif args.workload == "batched":
        prec = args.precision or "fp32"
        api.load_batched_tuning_file(os.path.join(ROOT, "paper_2310_20285_amd",
                                                  "batched_tuning_gfx950.json"))
        ws_ = datagen.config4()
        ms = [api.IterNCGP(torch.tensor(w.X, dtype=torch.float32, device="cuda"),
                           torch.tensor(w.y, dtype=torch.int32, device="cuda"), w.C, w.kernel,
                           w.lengthscale, w.outputscale, policy="cg", j_max=200,
                           rank_limit=100, recycle=True, precision=prec,
                           residual_mode="recurrence", max_buffer=300) for w in ws_]
        buf = None
        steps = min(args.reps, 3)
        iters = []
        for _ in range(steps):
            infos, buf = api.newton_step_batched(ms, buf)
            iters.append(sum(i["iters"] for i in infos))
        what = (f"{steps} batched Newton steps over {len(ms)} problems ({prec}; solver "
                f"iterations {iters})")
    else:
        prec = args.precision or "fp32"
        w = datagen.config5_model()
        X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
        y = torch.tensor(w.y, dtype=torch.int32, device="cuda")
        m = api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="cg",
                         j_max=100, rank_limit=100, precision=prec, residual_mode="recurrence",
                         max_buffer=200)
        for _ in range(3):
            m.newton_step()
        kept = m.compress(100)
        Xs = torch.tensor(np.random.default_rng(9).standard_normal((4096, w.D)),
                          dtype=torch.float32, device="cuda")
        ws = torch.empty(m.predict_ws_bytes(4096), dtype=torch.uint8, device="cuda")
        o = torch.empty((3, 4096 * w.C), dtype=torch.float32, device="cuda")
        st = torch.cuda.current_stream()
        for _ in range(args.reps):
            m.predict_into(Xs, o[0], o[1], o[2], ws, st)
        what = f"{args.reps} predictions at 4096 points (N={w.N}, C={w.C}, B={kept}, {prec})"
    torch.cuda.synchronize()
    n = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profile_driver: {what} and one {args.copy_mib} MiB device copy done")


if __name__ == "__main__":
    main()
