"""Profiling driver for rocprofv3.

    python -m paper_2310_20285_amd.profile_driver [--reps 20] [--copy-mib 256]

Runs the fused K.v product of the benchmark workload (N=20000, D=16, C=5,
Matern-5/2, FP32; the product the Newton step issues) ``--reps`` times via
glm_kernel_matmul, then one device-to-device copy of ``--copy-mib`` MiB.  The
copy is a transfer of known size: its FETCH_SIZE / WRITE_SIZE readings give
the factor that converts the counters of the K.v kernel to bytes.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    args = ap.parse_args()

    import torch

    import datagen
    from paper_2310_20285_amd import api

    w = datagen.config2()
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
    v = torch.randn(w.N * w.C, dtype=torch.float32, device="cuda")
    out = None
    for _ in range(args.reps):
        out = api.glm_kernel_matmul(X, X, v, w.C, w.kernel, w.lengthscale, w.outputscale,
                                    args.precision, out=out)
    torch.cuda.synchronize()
    n = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profile_driver: {args.reps} K.v products (N={w.N}, D={w.D}, C={w.C}) and one "
          f"{args.copy_mib} MiB device copy done")


if __name__ == "__main__":
    main()
