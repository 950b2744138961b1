#!/usr/bin/env python3
"""IterNCGP Newton steps per second on one MI355X.

Workload (N=20000, D=16, C=5): X ~ N(0, I_16), labels from the softmax of a
GP draw, Matern-5/2 prior (lengthscale 2, outputscale 1); IterNCGP-CG with
residual actions, at most 200 new actions per Newton step, compression to
R=100 eigenpairs at every virtual solver run, FP32 matrix-free K products and
FP64 reductions / projected solves.  One timed step = one Newton step
(Algorithms 1-3) followed by the prediction (mean, variance, probit) at the
2000 test points.  Inputs are seeded and synthetic and resident in HBM before
timing starts.

The timed region is the first ``--steps`` Newton steps of a fresh fit
(f_0 = 0, empty buffers); a separate model instance is warmed up first.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build measures one
GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Issue-bound ("alu") roofline of the fused FP32 product at small D.  FP32 MFMA
# and VALU work never execute at the same time on a
# SIMD, so one 16 x 16 block of kernel values on one wave costs the sum of its
# issue cycles:
#   full-rate FP32 VALU op   4 cycles (16 lanes per cycle, wave64; no packed FP32)
#   v_exp_f32 / v_sqrt_f32   8 cycles (measured: half the full rate)
#   v_mfma_f32_16x16x4f32   32 cycles (2048 flops at the 157.3 TFLOP/s FP32 matrix peak)
# A block is 4 values per lane x (transform + W multiply-adds) on VALU and the
# distance on 4 ceil(D/16) MFMAs; the symmetric kernel adds 4 MFMAs for the
# transposed sum, and then each evaluation serves two outputs.
SIMDS, CLOCK_HZ = 256 * 4, 2.4e9
VALU_CYCLES, TRANS_CYCLES, MFMA_F32_CYCLES = 4.0, 8.0, 32.0
# transform (full-rate, transcendental) per value, the distance add and scale
# included: Matern-3/2 and -5/2 take |t| into the square root as a free operand
# modifier, Matern-1/2 clamps t at 0 with one max
TRANSFORM_OPS = {"rbf": (2, 1), "matern12": (3, 2), "matern32": (4, 2), "matern52": (5, 2)}
KV_INSTANCE = None
# The solver products are timed with HIP events on the model's stream; each
# event pair costs a few microseconds of stream time (about 4% of a 230 us
# product), so every KV_SAMPLE-th product of the timed fit is bracketed and the
# average taken over those.
KV_SAMPLE = 3


# Bytes beyond L2 per launch of the product, from two rocprofv3 --pmc runs
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors read off a 256 MiB device
# copy in the same run; profiles/kv_matern52_N20000_D16_C5_fp32.md and
# profiles/kv_bf16_rbf_N60000_D784_C10.md).  Keyed by the kernel instance it
# was measured on; any other instance reports null.
MEASURED_TRAFFIC = {("kv_mfma_f32_sym<3,1,5,false>", "fp32"): 46.03e6,
                    # one prediction at 4096 points on the served model (variance
                    # pass kv_mfma_f32<0,2,4> 5.81 GB + mean pass 0.17 GB;
                    # profiles/predict_rbf_N100000_D32_C10_B100_fp32.md)
                    ("predict_4096_rbf_N100000_D32_C10_B100", "fp32"): 5.98e9,
                    # the symmetric BF16 product at N=60000 D=784 C=10, pairs in bands
                    # of 16 blocks (profiles/kv_bf16_rbf_N60000_D784_C10.md)
                    ("kv_bf16_sym<0, false>", "bf16"): 7.52e9}


def block_cycles(kind: str, W: int, D: int, symmetric: bool) -> float:
    full, trans = TRANSFORM_OPS[kind]
    valu = 4 * ((full + W) * VALU_CYCLES + trans * TRANS_CYCLES)
    mfma = (4 * math.ceil(D / 16) + (4 if symmetric else 0)) * MFMA_F32_CYCLES
    return valu + mfma


def peak_evals_per_s(kind: str, W: int, D: int, symmetric: bool) -> float:
    return SIMDS * CLOCK_HZ * 256 / block_cycles(kind, W, D, symmetric)


def cpu_baseline(w, k_products_per_step: float):
    """Time the oracle's FP64 K.v product on a bounded slice of the workload."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import kernels as ok
    rows = 4000
    rng = np.random.default_rng(0)
    v = rng.standard_normal((w.N, w.C))
    t0 = time.perf_counter()
    ok.kernel_matvec(w.X[:rows], w.X, v, w.kernel, w.lengthscale, w.outputscale)
    dt = time.perf_counter() - t0
    per_product = dt * (w.N / rows)
    per_step = per_product * k_products_per_step
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    # the same on one thread (BLAS pool limited to 1), on a quarter of the rows
    rows1 = rows // 4
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ok.kernel_matvec(w.X[:rows1], w.X, v, w.kernel, w.lengthscale, w.outputscale)
        dt1 = time.perf_counter() - t0
    per_product1 = dt1 * (w.N / rows1)
    return {"value": 1.0 / per_step, "unit": "Newton steps/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"oracle.kernels.kernel_matvec (FP64 numpy) on {rows} of the {w.N} rows "
                       f"of one K.v product ({dt:.1f} s), scaled to a full product "
                       f"({per_product:.1f} s) and to {k_products_per_step:.0f} products per "
                       f"Newton step as measured on the GPU; elementwise numpy runs on one "
                       f"thread, its matrix products on the BLAS pool"),
            "single_thread": {"value": 1.0 / (per_product1 * k_products_per_step),
                              "unit": "Newton steps/s", "cores": 1,
                              "sample": f"{rows1} rows ({dt1:.1f} s), scaled the same way"}}


FIT_STEPS = 5            # Newton steps per fit of the default schedule
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 peak (vector and matrix)


def golden(name: str) -> dict:
    """Stored FP64 reference values (written by tests/golden/make_fullsize_golden.py
    from the oracle alone)."""
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        return json.load(f)


def rel_err(a, b) -> float:
    import numpy as np
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--residual", default="recurrence", choices=["explicit", "recurrence"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain FP32 PyTorch comparison")
    ap.add_argument("--no-headline", action="store_true",
                    help="default workload: skip the BF16 image product and the serving p99")
    ap.add_argument("--precision", default=None, choices=["fp32", "fp64", "bf16", "bf16x3"])
    ap.add_argument("--workload", default="gpc16",
                    choices=["gpc16", "image", "batched", "serving", "gmm", "poisson", "peaks",
                             "perclass"],
                    help="gpc16: N=20000 D=16 C=5 (default); image: N=60000 D=784 C=10 BF16; "
                         "batched: 64 independent problems in one persistent launch; "
                         "serving: request stream against a fitted N=100000 D=32 C=10 model; "
                         "gmm: the paper's Gaussian-mixture classification (N=100000, D=3, "
                         "C=10); poisson: the paper's Poisson budget-split schedules; "
                         "peaks: issue-rate microbenchmarks behind the ALU roofline")
    ap.add_argument("--requests", type=int, default=160, help="serving: stream length")
    ap.add_argument("--tuning-file", default=os.path.join(ROOT, "paper_2310_20285_amd",
                                                          "batched_tuning_gfx950.json"),
                    help="batched: launch-shape table to seed the tuner from (if present)")
    ap.add_argument("--retune", action="store_true",
                    help="batched: ignore the table file and time every shape")
    ap.add_argument("--save-tuning", action="store_true",
                    help="batched: write the table (loaded and newly timed entries) to the file")
    ap.add_argument("--device-control", action="store_true",
                    help="batched: also time the steps with the control flow on the device")
    ap.add_argument("--load", type=float, nargs="+", default=[0.5],
                    help="serving: arrival rates as fractions of the measured capacity")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    from paper_2310_20285_amd import api

    dev = torch.device("cuda:0")
    global KV_INSTANCE
    if args.workload == "image":
        return print(json.dumps(bench_image(args)))
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "serving":
        return print(json.dumps(bench_serving(args)))
    if args.workload == "gmm":
        return bench_gmm(args)
    if args.workload == "poisson":
        return bench_poisson(args)
    if args.workload == "peaks":
        return bench_peaks(args)
    if args.workload == "perclass":
        return bench_perclass(args)
    args.precision = args.precision or "fp32"
    KV_INSTANCE = "kv_mfma_f32_sym<3,1,5,false>"   # Matern-5/2, D <= 16, W = 5, shared kernel
    w = datagen.config2()
    dt = torch.float64 if args.precision == "fp64" else torch.float32
    X = torch.tensor(w.X, dtype=dt, device=dev)
    y = torch.tensor(w.y, dtype=torch.int32, device=dev)
    Xs = torch.tensor(w.Xs, dtype=dt, device=dev)
    jmax, R = 200, 100

    def make_model():
        return api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="cg",
                            j_max=jmax, rank_limit=R, recycle=True, tol_abs=1e-5, tol_rel=1e-5,
                            precision=args.precision, residual_mode=args.residual,
                            max_buffer=jmax + R)

    # warm-up: a separate model runs up to one fit's Newton steps + predictions
    mw = make_model()
    for _ in range(min(args.warmup, FIT_STEPS)):
        mw.newton_step()
        mw.predict(Xs)
    torch.cuda.synchronize()
    del mw
    # timed: whole fresh fits of FIT_STEPS Newton steps from f_0 = 0 (empty
    # buffers), each step followed by the prediction at the test points, repeated
    # until `steps` Newton steps are timed; each fit's model is created before its
    # timed segment, and the segments are summed
    elapsed = 0.0
    infos, fit_iters, pred_ev = [], [], []
    prof = {}
    check = None            # the first fit's model, kept for the error check
    done = 0
    # prediction outputs are allocated once; the workspace grows with the fit's
    # buffer columns and is reallocated (doubled) only when the query exceeds it
    n_s = Xs.shape[0]
    pout = torch.empty((3, n_s * w.C), dtype=dt, device=dev)
    pws = None
    st = torch.cuda.current_stream()
    while done < args.steps:
        m = make_model()
        m.set_profiling(True, every=KV_SAMPLE)
        n_here = min(FIT_STEPS, args.steps - done)
        events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(n_here)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for a, b in events:
            info = m.newton_step()
            infos.append(info)
            its.append(info["iters"])
            need = m.predict_ws_bytes(n_s)
            if pws is None or pws.numel() < need:
                pws = torch.empty(2 * need, dtype=torch.uint8, device=dev)
            a.record()
            m.predict_into(Xs, pout[0], pout[1], pout[2], pws, st)
            b.record()
            pred_ev.append((a, b))   # read after the loop: the next step queues behind it
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        done += n_here
        fit_iters.append(its)
        for k, v in m.profile().items():
            prof[k] = prof.get(k, 0) + v
        if check is None:
            check = (m, n_here)
        else:
            del m
    pred_ms = [a.elapsed_time(b) for a, b in pred_ev]

    value = args.steps / elapsed
    launches = max(prof["kv_launches"], 1)
    kv_avg_s = prof["kv_ms"] / launches / 1e3
    symmetric = prof["kv_symmetric"] == prof["kv_launches"] > 0
    evals_per_launch = prof["kv_evals"] / launches
    achieved_evals = evals_per_launch / kv_avg_s
    peak_evals = peak_evals_per_s(w.kernel, w.C, w.D, symmetric)
    dense_flops = 2.0 * w.N * w.N * (w.D + w.C)          # 2 N1 N2 (D + W) per product
    method_flops = prof["kv_flops"] / launches            # what the kernel that ran evaluates
    achieved = dense_flops / kv_avg_s / 1e12
    k_per_step = sum(i["k_products"] for i in infos) / max(len(infos), 1)
    total_iters = sum(i["iters"] for i in infos)
    sched = fit_iters[0]

    out = {
        "metric": "IterNCGP Newton steps/s",
        "value": value,
        "unit": "Newton steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16", "bf16x3": "bf16x3"}[
            args.precision],
        "data": "synthetic",
        "config": {"workload": (f"gpc N=20000 D=16 C=5 matern52 l=2; IterNCGP-CG j<=200 R=100, "
                                f"tol 1e-5; {len(fit_iters)} fresh fit(s) of {FIT_STEPS} Newton "
                                f"steps from f_0=0 ({args.steps} steps timed; solver "
                                f"iterations per step of a fit: {sched}), each step followed "
                                f"by predict (mean, variance, probit) at 2000 test points"),
                   "residual": args.residual,
                   "N": w.N, "D": w.D, "C": w.C, "j_max": jmax, "rank_limit": R,
                   "precision": args.precision, "test_points": int(Xs.shape[0]),
                   "fits": len(fit_iters), "steps_per_fit": FIT_STEPS},
        "solver_iterations": {"total": total_iters, "per_s": total_iters / elapsed,
                              "ms_per_iteration": elapsed / max(total_iters, 1) * 1e3,
                              "per_fit": fit_iters},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": MEASURED_TRAFFIC.get((KV_INSTANCE, args.precision)),
                     "kernel": ("symmetric fused K.v (each pair of rows evaluated once)"
                                if symmetric else "fused K.v"),
                     "flops_per_launch": dense_flops,
                     "flop_count": "2 N1 N2 (D + W) per product, W = C output columns",
                     "avg_launch_us": kv_avg_s * 1e6,
                     "method_flops_per_launch": method_flops,
                     "frac_method_flops": method_flops / kv_avg_s / 1e12 / FP32_PEAK_TFLOPS,
                     "issue_model": {"achieved_geval_s": achieved_evals / 1e9,
                                     "peak_geval_s": peak_evals / 1e9,
                                     "frac": achieved_evals / peak_evals,
                                     "cycles": {"valu": VALU_CYCLES, "transcendental":
                                                TRANS_CYCLES, "mfma_f32": MFMA_F32_CYCLES}}},
        "kv": {"launches_timed": prof["kv_launches"], "timed_every": KV_SAMPLE,
               "avg_us": kv_avg_s * 1e6, "k_products_per_step": k_per_step,
               "share_of_step": kv_avg_s * 1e3 * k_per_step * len(infos)
                                / max(prof["step_ms"], 1e-9)},
        "predict_latency_ms": {"p50": float(np.percentile(pred_ms, 50)),
                               "p99": float(np.percentile(pred_ms, 99)),
                               "timing": "HIP events around each call on the model's stream"},
        "newton": [{k: (round(v, 6) if isinstance(v, float) else v) for k, v in i.items()
                    if k in ("iters", "buffer_cols", "converged", "res_norm", "rel_change", "psi")}
                   for i in infos[:FIT_STEPS]],
    }
    out["error_vs_fp64"] = fp64_error_default(w, check[0], check[1], Xs)
    del check
    if not args.no_plain:
        out["plain_fp32"] = plain_comparison(w, X, y, Xs, sched, R, out)
        out["dense_k_fp32"] = dense_k(w, X, kv_avg_s)
    if not args.no_headline:
        out["headline"] = {"bf16_image_product": bf16_product_headline(),
                           "serving_p99": serving_headline(args)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, k_per_step)
    print(json.dumps(out))


def fp64_error_default(w, m, steps_done, Xs):
    """The fit against the FP64 O-method reference of the same schedule (the
    oracle's Algorithms 1-3 on the CPU, stored values): Newton iterate f at 256
    stored rows after the last step, predictive mean at 256 test points after a
    whole fit, iteration counts."""
    import numpy as np
    g = golden("omethod_config2.json")
    rows = np.asarray(g["rows"])
    F = m.view(0).double().cpu().numpy().reshape(w.N, w.C)
    ref = g["steps"][steps_done - 1]
    res = {"reference": "FP64 O-method (Algorithms 1-3 on the CPU, stored by "
                        "tests/golden/make_fullsize_golden.py)",
           "after_step": steps_done,
           "f_rel_err_256_rows": rel_err(F[rows], ref["F_rows"]),
           "iters_fp64": [s["iters"] for s in g["steps"][:steps_done]]}
    if steps_done == len(g["steps"]):
        mean, _, _ = m.predict(Xs[:g["test_points"]], var=False, probs=False)
        res["pred_mean_rel_err_256_points"] = rel_err(mean.double().cpu().numpy(), g["mean"])
    return res


def dense_k(w, X, fused_s):
    """Dense-K-in-HBM FP32 product (K formed once, then one GEMM per product)
    beside the fused product's time."""
    from plain_fp32 import dense_k_comparison
    r = dense_k_comparison(X, w.C, w.kernel, w.lengthscale, w.outputscale)
    if "product_ms" in r:
        r["fused_product_ms"] = fused_s * 1e3
        r["dense_over_fused"] = r["product_ms"] / (fused_s * 1e3)
    return r


def plain_comparison(w, X, y, Xs, sched, R, ours):
    """The plain FP32 PyTorch form on the same GPU at equal solver work: one fit
    with the library's per-step iteration counts imposed (tolerance 0), each
    step followed by the prediction; per Newton step, per solver iteration, per
    product with K and per prediction (both timed with device events)."""
    import numpy as np
    import torch

    from plain_fp32 import PlainIterNCGP
    pm = PlainIterNCGP(X.float(), y, w.C, w.kernel, w.lengthscale, w.outputscale,
                       j_max=max(sched + [1]), rank_limit=R, tol_abs=0.0, tol_rel=0.0)
    torch.cuda.synchronize()
    lat = []
    its = []
    t0 = time.perf_counter()
    for j in sched:
        its.append(pm.newton_step(j_max=j)["iters"])
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        pm.predict(Xs.float())
        b.record()
        b.synchronize()
        lat.append(a.elapsed_time(b))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / len(sched)
    # one product with K, timed alone
    v = torch.randn(w.N * w.C, device=X.device)
    pm.apply_K(v)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        pm.apply_K(v)
    e1.record()
    e1.synchronize()
    kv_ms = e0.elapsed_time(e1) / 5
    ours_step_ms = ours["ms_per_step"]
    ours_it_ms = ours["solver_iterations"]["ms_per_iteration"]
    it_ms = dt * 1e3 * len(sched) / max(sum(its), 1)
    p99 = float(np.percentile(lat, 99))
    return {"value": 1.0 / dt, "unit": "Newton steps/s", "ms_per_step": dt * 1e3,
            "schedule": "the library's solver iterations per step imposed, tolerance 0",
            "iters_per_step": its,
            "speedup_of_library_per_step": dt * 1e3 / ours_step_ms,
            "ms_per_solver_iteration": it_ms,
            "speedup_of_library_per_solver_iteration": it_ms / ours_it_ms,
            "kv_product_ms": kv_ms,
            "speedup_of_library_per_product": kv_ms / (ours["kv"]["avg_us"] / 1e3),
            "predict_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": p99},
            "p99_ratio_plain_over_library": p99 / ours["predict_latency_ms"]["p99"]}


def bf16_product_headline() -> dict:
    """The image-shaped product (N=60000, D=784, C=10, RBF, median lengthscale)
    through glm_kernel_matmul in both BF16 modes: device time (HIP events on
    the calling stream, 5 calls; each call prepares the rows, runs the
    symmetric product and reduces its partials), TFLOP/s against the BF16
    matrix peak, and the error against stored FP64 values of 64 rows."""
    import numpy as np
    import torch

    import datagen
    from paper_2310_20285_amd import api
    w = datagen.config3(Ns=1000)        # the lengthscale depends on the draw of test points
    g = golden("kv_products.json")["config3"]
    assert abs(w.lengthscale - g["lengthscale"]) <= 1e-12 * g["lengthscale"]
    rng = np.random.default_rng(2024)
    v = rng.standard_normal(w.N * w.C).astype(np.float32)
    X = torch.tensor(w.X, dtype=torch.float32, device="cuda")
    vd = torch.tensor(v, device="cuda")
    rows = np.asarray(g["rows"])
    method = w.N * (w.N + 1.0) * w.D + 2.0 * w.N * w.N * w.C   # each pair once
    dense = 2.0 * w.N * w.N * (w.D + w.C)
    res = {"workload": "image-shaped N=60000 D=784 C=10 rbf, one vector (W=10)",
           "flop_count": "method N(N+1) D + 2 N^2 W (each pair of rows once); dense "
                         "2 N^2 (D + W)"}
    for mode in ("bf16", "bf16x3"):
        out = api.glm_kernel_matmul(X, X, vd, w.C, w.kernel, w.lengthscale, w.outputscale, mode)
        err = rel_err(out.double().cpu().numpy().reshape(w.N, w.C)[rows], g["ref"])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            api.glm_kernel_matmul(X, X, vd, w.C, w.kernel, w.lengthscale, w.outputscale, mode,
                                  out=out)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 5
        res[mode] = {"ms": ms, "tflops_method": method / ms / 1e9,
                     "frac_bf16_peak_method": method / ms / 1e9 / BF16_MFMA_PEAK_TFLOPS,
                     "frac_bf16_peak_dense": dense / ms / 1e9 / BF16_MFMA_PEAK_TFLOPS,
                     "frac_measured_random_operand_rate_method":
                         method / ms / 1e9 / BF16_MFMA_RANDOM_TFLOPS,
                     "rel_err_vs_fp64_64_rows": err}
    return res


def serving_headline(args) -> dict:
    """p99 of the predictive queries in a shortened serving stream (100
    requests at half the measured capacity) against the fitted N=100000 model."""
    a = argparse.Namespace(**vars(args))
    a.requests, a.load, a.no_plain, a.precision = 100, [0.5], True, "fp32"
    r = bench_serving(a)
    run = r["runs"][0]
    return {"p99_ms": r["value"], "p50_ms": run["predict"].get("p50_ms"),
            "capacity_rps": r["capacity_rps"], "requests": r["config"]["requests"],
            "alone_vs_mix_mismatches": r["alone_vs_mix_mismatches"],
            "workload": r["config"]["workload"]}


def bench_batched(args):
    """64 independent problems (N ~ U{1000..16000}, D=8, C ~ U{2..8},
    Matern-3/2), IterNCGP-CG j<=200, R=100, FP32: one batched Newton step over
    all problems per step (one persistent launch per solver iteration),
    against the same steps run problem by problem with the library and with
    the plain FP32 form.  value = aggregate Newton steps/s (problems x steps /
    time)."""
    import torch

    import datagen
    from paper_2310_20285_amd import api

    prec = args.precision or "fp32"
    if prec not in ("fp32", "bf16"):
        raise SystemExit("the batched form takes FP32 or BF16 models")
    ws_ = datagen.config4()
    dev = torch.device("cuda:0")
    data = [(torch.tensor(w.X, dtype=torch.float32, device=dev),
             torch.tensor(w.y, dtype=torch.int32, device=dev)) for w in ws_]
    steps = max(1, min(args.steps, 3))

    def models():
        return [api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="cg",
                             j_max=200, rank_limit=100, recycle=True, precision=prec,
                             residual_mode="recurrence", max_buffer=300)
                for w, (X, y) in zip(ws_, data)]

    # the launch-shape table: seeded from the saved file (shapes it covers skip
    # the timing), or timed afresh and saved with --retune
    seeded = 0
    if not args.retune and os.path.exists(args.tuning_file):
        seeded = api.load_batched_tuning_file(args.tuning_file)
    # warm-up (also runs the launch-shape tuning of shapes the table lacks)
    wm = models()
    buf = None
    _, buf = api.newton_step_batched(wm, buf)
    del wm
    torch.cuda.synchronize()
    ms = models()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(steps):
        infos, buf = api.newton_step_batched(ms, buf)
        iters.append(sum(i["iters"] for i in infos))
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    del ms
    # the same with the control flow on the device (windows of iterations), on request
    dc_line = None
    if args.device_control:
        ms = models()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters_dc = []
        for _ in range(steps):
            infos, buf = api.newton_step_batched(ms, buf, device_control=True)
            iters_dc.append(sum(i["iters"] for i in infos))
        torch.cuda.synchronize()
        t_dc = time.perf_counter() - t0
        del ms
        dc_line = {"value": len(ws_) * steps / t_dc, "unit": "Newton steps/s",
                   "ms_per_step": t_dc / steps * 1e3,
                   "speedup_over_host_control": t_batch / t_dc,
                   "solver_iterations_per_batched_step": iters_dc}
    ms = models()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for m in ms:
            m.newton_step()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    del ms
    res = {
        "metric": "IterNCGP Newton steps/s (aggregate over problems)",
        "value": len(ws_) * steps / t_batch,
        "unit": "Newton steps/s",
        "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": t_batch / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16"}[prec], "data": "synthetic",
        "config": {"workload": "64 problems N~U{1000..16000} D=8 C~U{2..8} matern32; "
                               "IterNCGP-CG j<=200 R=100; batched Newton steps",
                   "precision": prec,
                   "problems": len(ws_), "sum_N": int(sum(w.N for w in ws_))},
        "solver_iterations_per_batched_step": iters,
        "device_control": dc_line,
        "sequential_library": {"value": len(ws_) * steps / t_seq, "unit": "Newton steps/s",
                               "speedup_of_batched": t_seq / t_batch},
        "tuning": json.loads(api.batched_tuning()),
        "tuning_seeded_from_file": seeded,
    }
    if args.save_tuning:
        api.save_batched_tuning_file(args.tuning_file)
        res["tuning_saved_to"] = os.path.relpath(args.tuning_file, ROOT)
    if not args.no_plain:
        from plain_fp32 import PlainIterNCGP
        pms = [PlainIterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, j_max=200,
                             rank_limit=100) for w, (X, y) in zip(ws_, data)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for pm in pms:
                pm.newton_step()
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        res["plain_fp32_sequential"] = {"value": len(ws_) * steps / t_plain,
                                        "unit": "Newton steps/s",
                                        "speedup_of_batched": t_plain / t_batch}
    print(json.dumps(res))


BF16_MFMA_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak
# v_mfma_f32_16x16x32_bf16 on random operands, measured by --workload peaks
# (19.7 cycles per instruction at 2.4 GHz): the matrix rate on data like the
# product's, which draws more power than the constant operands a peak assumes
BF16_MFMA_RANDOM_TFLOPS = 2041.0


def bench_image(args):
    """Image-shaped workload: N=60000, D=784, C=10, RBF (median lengthscale),
    BF16 distance GEMM (--precision bf16x3: the split-input mode).  IterNCGP-CG
    with j <= 5 per Newton step, no compression, 3 Newton steps (the paper's
    MNIST schedule), prediction at 1000 test points per step.  The fit is
    compared with the stored FP64 O-method run of the same schedule."""
    import numpy as np
    import torch

    import datagen
    from paper_2310_20285_amd import api

    prec = args.precision or "bf16"
    w = datagen.config3(Ns=1000)
    dev = torch.device("cuda:0")
    X = torch.tensor(w.X, dtype=torch.float32, device=dev)
    y = torch.tensor(w.y, dtype=torch.int32, device=dev)
    Xs = torch.tensor(w.Xs, dtype=torch.float32, device=dev)
    steps = min(args.steps, 3)

    def make_model():
        return api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="cg",
                            j_max=5, rank_limit=-1, recycle=True, precision=prec,
                            residual_mode=args.residual, max_buffer=5 * 3 + 1)

    mw = make_model()
    mw.newton_step()
    torch.cuda.synchronize()
    del mw
    m = make_model()
    m.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        infos.append(m.newton_step())
        m.predict(Xs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = m.profile()
    kv_avg_s = prof["kv_ms"] / max(prof["kv_launches"], 1) / 1e3
    # algorithmic flops of the method that ran: n(n+1) D + 2 n^2 C for the
    # symmetric product (each pair of rows once), 2 n^2 (D + C) one-sided
    symmetric = prof["kv_symmetric"] == prof["kv_launches"] > 0
    flops = prof["kv_flops"] / max(prof["kv_launches"], 1)
    tflops = flops / kv_avg_s / 1e12
    dense_tflops = 2.0 * w.N * w.N * (w.D + w.C) / kv_avg_s / 1e12
    # the fit against the stored FP64 O-method run (F at 256 rows after each
    # step, predictive mean at 256 test points after the last)
    g = golden("omethod_config3.json")
    rows = np.asarray(g["rows"])
    F = m.view(0).double().cpu().numpy().reshape(w.N, w.C)
    err = {"reference": "FP64 O-method (Algorithms 1-3 on the CPU, stored)",
           "after_step": steps,
           "f_rel_err_256_rows": rel_err(F[rows], g["steps"][steps - 1]["F_rows"])}
    if steps == len(g["steps"]):
        mean, _, _ = m.predict(Xs[:g["test_points"]], var=False, probs=False)
        err["pred_mean_rel_err_256_points"] = rel_err(mean.double().cpu().numpy(), g["mean"])
    # one product against stored FP64 values at 64 rows
    gp = golden("kv_products.json")["config3"]
    assert abs(w.lengthscale - gp["lengthscale"]) <= 1e-12 * gp["lengthscale"]
    v = np.random.default_rng(2024).standard_normal(w.N * w.C).astype(np.float32)
    out = api.glm_kernel_matmul(X, X, torch.tensor(v, device=dev), w.C, w.kernel,
                                w.lengthscale, w.outputscale, prec).double().cpu().numpy()
    err["kv_rel_err_64_rows"] = rel_err(out.reshape(w.N, w.C)[np.asarray(gp["rows"])], gp["ref"])
    instance = {"bf16": "kv_bf16_sym<0, false>", "bf16x3": "kv_bf16_sym<0, true>"}.get(prec)
    res = {
        "metric": "IterNCGP Newton steps/s",
        "value": steps / (t1 - t0),
        "unit": "Newton steps/s",
        "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": (t1 - t0) / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": "image-shaped N=60000 D=784 C=10 rbf (median lengthscale); "
                               "IterNCGP-CG j<=5 R=inf, 3 Newton steps, predict 1000 test points",
                   "lengthscale": w.lengthscale, "zero_frac": w.meta.get("zero_frac"),
                   "precision": prec, "residual": args.residual},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": BF16_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / BF16_MFMA_PEAK_TFLOPS,
                     "traffic": MEASURED_TRAFFIC.get((instance, prec)) if symmetric else None,
                     "kernel": ("symmetric fused K.v, BF16 distance GEMM (N(N+1) D + 2 N^2 C "
                                "flops per product)" if symmetric else
                                "fused K.v, BF16 distance GEMM (2 N^2 (D + C) flops per product)"),
                     "avg_launch_us": kv_avg_s * 1e6,
                     "dense_equivalent_tflops": dense_tflops,
                     "frac_measured_random_operand_rate": tflops / BF16_MFMA_RANDOM_TFLOPS},
        "error_vs_fp64": err,
        "dense_k_fp32": None if args.no_plain else dense_k(w, X, kv_avg_s),
        "newton": [{k: (round(v_, 6) if isinstance(v_, float) else v_) for k, v_ in i.items()
                    if k in ("iters", "buffer_cols", "rel_change", "psi")} for i in infos],
    }
    return res


FP32_MFMA_PEAK_TFLOPS = 157.3   # MI355X dense FP32 matrix peak


def bench_serving(args):
    """Serving workload.  Fitted model: N=100000, D=32, C=10, RBF (lengthscale
    sqrt(2D), outputscale 1), IterNCGP-CG j<=100, R=100, 3 Newton steps, then
    compressed to B=100 directions (Algorithm 3).  Stream: Poisson arrivals,
    95% predictive queries of ceil(exp(U(0, ln 4096))) test points, 5% new fits
    with N ~ U{2000..50000} (j<=50, R=50, 2 Newton steps), HBM budget 8 GB.

    capacity = requests/s with the whole stream submitted at once.  The stream
    is then replayed in real time at each --load fraction of that capacity, by
    the continuous-batching server and by the plain FP32 form serving the same
    fitted state one request at a time (FIFO).  value = p99 latency of the
    predictive queries at the first --load fraction."""
    import numpy as np
    import torch

    import datagen
    from paper_2310_20285_amd import api
    from paper_2310_20285_amd.serving import Server, latency_stats

    prec = args.precision or "fp32"
    dev = torch.device("cuda:0")
    w = datagen.config5_model()
    X = torch.tensor(w.X, dtype=torch.float32, device=dev)
    y = torch.tensor(w.y, dtype=torch.int32, device=dev)
    B = 100
    m = api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="cg", j_max=100,
                     rank_limit=100, recycle=True, precision=prec, residual_mode="recurrence",
                     max_buffer=200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit_info = [m.newton_step() for _ in range(3)]
    kept = m.compress(B)
    fit_s = time.perf_counter() - t0

    fit_cfg = dict(policy="cg", j_max=50, rank_limit=50, recycle=True, precision=prec,
                   residual_mode="recurrence", max_buffer=100)
    reqs = datagen.config5_requests(n_requests=args.requests, rate_hz=100.0, D=w.D)
    for r in reqs:
        if r["kind"] == "fit":
            f = datagen.config5_fit(r["seed"], r["n"], D=w.D, C=w.C)
            r.update(X=f.X, y=f.y, C=w.C, kernel=f.kernel, lengthscale=f.lengthscale,
                     outputscale=f.outputscale)
    budget = 8 * 10**9

    def server():
        return Server(m, budget_bytes=budget, max_batch_rows=8192, slots=2, fit_workers=2,
                      fit_config=dict(fit_cfg, steps=2))

    # warm-up: a short stream through a server (kernels, allocator, threads)
    server().replay(reqs[:12], realtime=False)
    torch.cuda.synchronize()
    srv = server()
    tk = srv.replay(reqs, realtime=False)
    makespan = max(t.t_done for t in tk)
    capacity = len(reqs) / makespan
    n_fit = sum(1 for r in reqs if r["kind"] == "fit")
    pts = sum(r["X"].shape[0] for r in reqs if r["kind"] == "predict")

    def scaled(frac):
        scale = 100.0 / (frac * capacity)
        return [dict(r, t=r["t"] * scale) for r in reqs]

    runs = []
    for frac in args.load:
        srv = server()
        tk = srv.replay(scaled(frac), realtime=True)
        span = max(t.t_done for t in tk)
        runs.append({"load": frac, "rate_rps": frac * capacity,
                     "predict": latency_stats(tk, "predict"), "fit": latency_stats(tk, "fit"),
                     "refused": sum(1 for t in tk if t.status == "refused"),
                     "batches": srv.batches,
                     "mean_batch_rows": float(np.mean(srv.batch_rows)) if srv.batch_rows else 0.0,
                     "queries_per_s": (len(reqs) - n_fit) / span,
                     "test_points_per_s": pts / span,
                     "newton_steps_per_s": 2 * n_fit / span})
        if frac == args.load[0]:
            first = tk
            slow = sorted((t for t in tk if t.kind == "predict"), key=lambda t: -t.latency)[:5]
            runs[-1]["slowest_predicts"] = [
                {"rows": t.rows, "latency_ms": round(t.latency * 1e3, 2),
                 "queued_ms": round((t.t_start - t.t_arrive) * 1e3, 2),
                 "fits_running": sum(1 for f in tk if f.kind == "fit" and f.t_start <= t.t_done
                                     and f.t_done >= t.t_start)} for t in slow]
    # alone vs in the mix, on a few of the served queries (tolerance: bitwise)
    mism = 0
    for t in [t for t in first if t.kind == "predict"][:8]:
        mean, var, probs = m.predict(torch.tensor(t.payload["X"], device=dev))
        for key, ref in (("mean", mean), ("var", var), ("probs", probs)):
            mism += int(not np.array_equal(t.result[key], ref.cpu().numpy()))

    # the dominant kernel: K(X*, X) [v | Q] at 4096 test points
    Xs = torch.tensor(np.random.default_rng(9).standard_normal((4096, w.D)), dtype=torch.float32,
                      device=dev)
    ws = torch.empty(m.predict_ws_bytes(4096), dtype=torch.uint8, device=dev)
    out = torch.empty((3, 4096 * w.C), device=dev)
    st = torch.cuda.current_stream()
    for _ in range(2):
        m.predict_into(Xs, out[0], out[1], out[2], ws, st)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(st)
    reps = 10
    for _ in range(reps):
        m.predict_into(Xs, out[0], out[1], out[2], ws, st)
    ev[1].record(st)
    ev[1].synchronize()
    pred_ms = ev[0].elapsed_time(ev[1]) / reps
    flops = 2.0 * 4096 * w.N * (2 * w.D + w.C * (1 + kept))
    tflops = flops / (pred_ms / 1e3) / 1e12
    peak = FP32_MFMA_PEAK_TFLOPS if prec == "fp32" else BF16_MFMA_PEAK_TFLOPS

    res = {
        "metric": "p99 predict latency (served stream at %.2gx capacity)" % args.load[0],
        "value": runs[0]["predict"].get("p99_ms"),
        "unit": "ms",
        "n_gpus": 1, "steps": len(reqs), "warmup": 12,
        "ms_per_step": makespan / len(reqs) * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16"}[prec], "data": "synthetic",
        "config": {"workload": "serving: fitted N=100000 D=32 C=10 rbf, B=100; Poisson stream "
                               "95% predict (1..4096 points, log-uniform) / 5% fits "
                               "(N~U{2000..50000}, j<=50 R=50, 2 steps); HBM budget 8 GB",
                   "requests": len(reqs), "fits": n_fit, "test_points": pts,
                   "precision": prec, "budget_bytes": budget},
        "served_model": {"fit_s": fit_s, "kept_directions": kept,
                         "iters": [i["iters"] for i in fit_info]},
        "capacity_rps": capacity,
        "runs": runs,
        "alone_vs_mix_mismatches": mism,
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": tflops / peak,
                     "traffic": MEASURED_TRAFFIC.get(
                         ("predict_4096_rbf_N100000_D32_C10_B100", prec)) if kept == 100 else None,
                     "kernel": "prediction at 4096 points: K(X*,X) v and K(X*,X) Q "
                               "(2 N* N (2D + C(1+B)) flops)",
                     "avg_call_ms": pred_ms},
    }
    if not args.no_plain:
        from plain_fp32 import PlainIterNCGP, fifo_replay
        pm = PlainIterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale)
        pm.v = m.view(1).float()
        pm.Q = m.view(2).float().t().contiguous()
        pr = {}
        for frac in args.load[:1]:
            rec = fifo_replay(pm, scaled(frac), dict(j_max=50, rank_limit=50), 2)
            lat = np.array([d - a for k, a, d in rec if k == "predict"]) * 1e3
            flat = np.array([d - a for k, a, d in rec if k == "fit"]) * 1e3
            pr = {"load": frac, "predict": {"p50_ms": float(np.percentile(lat, 50)),
                                            "p99_ms": float(np.percentile(lat, 99))},
                  "fit": {"p50_ms": float(np.percentile(flat, 50)) if flat.size else None,
                          "p99_ms": float(np.percentile(flat, 99)) if flat.size else None},
                  "span_s": max(d for _, _, d in rec)}
        pr["p99_ratio_plain_over_library"] = pr["predict"]["p99_ms"] / res["value"]
        res["plain_fp32_fifo"] = pr
    return res


def bench_gmm(args):
    """The paper's large-scale classification workload: a 10-class Gaussian
    mixture in 3-D, N = 100000 training and 10000 test points, Matern-3/2
    (lengthscale 0.05, outputscale 0.05); IterNCGP-CG with j <= 5 actions per
    Newton step and recycling, R = inf and R = 10.  After every Newton step the
    probit predictions at the test points give accuracy and NLL; both are
    reported against the cumulative device time.  value = Newton steps/s of
    the R = inf run (predictions excluded)."""
    import numpy as np
    import torch

    import datagen
    from paper_2310_20285_amd import api

    prec = args.precision or "fp32"
    w = datagen.gmm()
    dev = torch.device("cuda:0")
    X = torch.tensor(w.X, dtype=torch.float32, device=dev)
    y = torch.tensor(w.y, dtype=torch.int32, device=dev)
    Xs = torch.tensor(w.Xs, dtype=torch.float32, device=dev)
    steps = max(args.steps, 10)
    runs = {}
    for R in (-1, 10):
        def make():
            return api.IterNCGP(X, y, w.C, w.kernel, w.lengthscale, w.outputscale, policy="cg",
                                j_max=5, rank_limit=R, recycle=True, precision=prec,
                                residual_mode="recurrence",
                                max_buffer=5 * steps + 5 if R < 0 else R + 5)
        mw = make()
        mw.newton_step()
        torch.cuda.synchronize()
        del mw
        m = make()
        torch.cuda.synchronize()
        t_solve = 0.0
        curve = []
        for i in range(steps):
            t0 = time.perf_counter()
            info = m.newton_step()
            t_solve += time.perf_counter() - t0
            _, _, probs = m.predict(Xs)
            p = probs.double().cpu().numpy()
            acc = float((p.argmax(1) == w.ys).mean())
            nll = float(-np.mean(np.log(np.maximum(p[np.arange(len(w.ys)), w.ys], 1e-300))))
            curve.append({"step": i + 1, "solve_s": round(t_solve, 4), "iters": info["iters"],
                          "buffer_cols": info["buffer_cols"], "accuracy": round(acc, 4),
                          "nll": round(nll, 4)})
        runs["R=inf" if R < 0 else f"R={R}"] = {"steps_per_s": steps / t_solve, "curve": curve}
    res = {
        "metric": "IterNCGP Newton steps/s",
        "value": runs["R=inf"]["steps_per_s"],
        "unit": "Newton steps/s",
        "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": 1e3 / runs["R=inf"]["steps_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[prec], "data": "synthetic",
        "config": {"workload": "Gaussian mixture N=100000 D=3 C=10 matern32 l=0.05 os=0.05; "
                               "IterNCGP-CG j<=5, recycling, R=inf and R=10; probit "
                               "predictions at 10000 test points after each step",
                   "precision": prec},
        "runs": runs,
    }
    print(json.dumps(res))


def bench_peaks(args):
    """Issue-rate microbenchmarks (libitergp_peaks.so): wave-instructions per
    SIMD per second of v_fma_f32, v_exp_f32, v_sqrt_f32 and the FP32 / BF16
    matrix instructions the product kernels use, expressed as cycles per
    instruction at the nominal 2.4 GHz, and whether FP32 MFMA and VALU work
    overlap (mixed loop time against the sum of the parts).  These are the
    constants of the ALU issue model of the default workload's roofline.
    Also the LDS read and write bandwidth (bytes per clock per CU, 16-byte
    accesses) and whether LDS reads overlap BF16 MFMAs, which bound the BF16
    product's feature loop."""
    import ctypes as ct

    import torch

    from paper_2310_20285_amd import build as pb
    lib = ct.CDLL(pb.PEAKS_LIB)
    lib.igp_peaks_run.restype = ct.c_int
    lib.igp_peaks_run.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_void_p,
                                  ct.c_void_p]
    blocks = 256 * 8                         # 8 workgroups of 4 waves per CU: 8 waves per SIMD
    waves_per_simd = blocks * 4 / SIMDS
    out = torch.empty(blocks * 256, device="cuda")
    st = torch.cuda.current_stream()

    def run(which, iters, nvalu=0):
        for rep in range(2):             # the first launch warms up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rc = lib.igp_peaks_run(which, blocks, iters, nvalu, ct.c_void_p(out.data_ptr()),
                                   ct.c_void_p(st.cuda_stream))
            e1.record()
            e1.synchronize()
            if rc != 0:
                raise RuntimeError(f"microbenchmark {which} failed ({rc})")
        return e0.elapsed_time(e1) / 1e3

    def cycles(t, per_trip, iters):
        instr = waves_per_simd * iters * per_trip          # wave-instructions per SIMD
        return t * CLOCK_HZ / instr

    it = 4000
    res = {}
    t_fma = run(0, it)
    res["v_fma_f32"] = {"cycles": cycles(t_fma, 64, it),
                        "tflops": 2 * 64 * waves_per_simd * SIMDS * it * 64 / t_fma / 1e12}
    res["v_exp_f32"] = {"cycles": cycles(run(1, it), 64, it)}
    res["v_sqrt_f32"] = {"cycles": cycles(run(2, it), 64, it)}
    t_mf = run(3, it)
    res["v_mfma_f32_16x16x4f32"] = {"cycles": cycles(t_mf, 16, it),
                                    "tflops": 2 * 16 * 16 * 4 * 16 * waves_per_simd * SIMDS * it
                                    / t_mf / 1e12}
    t_bf = run(4, it)
    res["v_mfma_f32_16x16x32_bf16"] = {"cycles": cycles(t_bf, 16, it),
                                       "tflops": 2 * 16 * 16 * 32 * 16 * waves_per_simd * SIMDS
                                       * it / t_bf / 1e12}
    t_bfr = run(8, it)
    res["v_mfma_f32_16x16x32_bf16_random_operands"] = {
        "cycles": cycles(t_bfr, 16, it),
        "tflops": 2 * 16 * 16 * 32 * 16 * waves_per_simd * SIMDS * it / t_bfr / 1e12}
    mixed = {}
    for nv in (32, 64, 128):
        t_mix = run(5, it, nv)
        t_valu = t_fma * nv / 64             # the same FMAs alone (kind 0 at the same count)
        mixed[str(nv)] = {"mixed_ms": t_mix * 1e3, "mfma_alone_ms": t_mf * 1e3,
                          "valu_alone_ms": t_valu * 1e3,
                          "overlap": (t_mf + t_valu - t_mix) / min(t_mf, t_valu)}
    res["mfma_f32_with_valu"] = mixed
    # the same two kinds in different waves of one SIMD (waves 0-3 MFMA, 4-7 FMA)
    split = {}
    t_sm = run(9, it, -1)                   # MFMA waves alone
    t_sv = run(9, it, -2)                   # FMA waves alone (64 FMAs per trip)
    for nv in (32, 64, 128):
        t_mix = run(9, it, nv)
        t_valu = t_sv * nv / 64
        split[str(nv)] = {"mixed_ms": t_mix * 1e3, "mfma_waves_alone_ms": t_sm * 1e3,
                          "fma_waves_alone_ms": t_valu * 1e3,
                          "overlap": (t_sm + t_valu - t_mix) / min(t_sm, t_valu)}
    res["mfma_f32_and_valu_in_different_waves"] = split
    # LDS: 8 ds_read_b128 per trip per wave (1 KB each), two 64 KB workgroups per CU
    lds_bytes = blocks * 4 * it * 8 * 1024

    def per_clk(t):                       # bytes per clock per CU
        return lds_bytes / (t * CLOCK_HZ * (SIMDS // 4))

    t_rd = {nm: run(6, it, nm) for nm in (4, 12, 24)}
    t_bf_one = t_bf / 16                  # time of one BF16 MFMA per wave at this launch
    lds = {"read_bytes_per_clk_per_cu": per_clk(t_rd[4]),
           "write_bytes_per_clk_per_cu": per_clk(run(7, it))}
    for nm in (12, 24):
        t_m = t_bf_one * nm
        lds[f"read_with_{nm}_bf16_mfma"] = {
            "mixed_ms": t_rd[nm] * 1e3, "lds_alone_ms": t_rd[4] * 1e3, "mfma_alone_ms": t_m * 1e3,
            "overlap": (t_rd[4] + t_m - t_rd[nm]) / min(t_rd[4], t_m)}
    res["lds"] = lds
    line = {"metric": "issue rates (cycles per wave-instruction per SIMD at 2.4 GHz)",
            "value": res["v_exp_f32"]["cycles"], "unit": "cycles per v_exp_f32",
            "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": None,
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": "issue-rate microbenchmarks, 8 waves per SIMD",
                       "blocks": blocks, "iters": it},
            "rates": res,
            "model_constants": {"valu": VALU_CYCLES, "transcendental": TRANS_CYCLES,
                                "mfma_f32": MFMA_F32_CYCLES}}
    print(json.dumps(line))


def bench_perclass(args):
    """Per-class kernels (one lengthscale and outputscale per latent function,
    the n_kp = C form of the product): at the default workload's shape (N =
    20000, D = 16, C = 5, Matern-5/2, lengthscales 1.5-2.5, outputscales
    0.8-1.2), the FP32 product K_c(X, X) v_c against the shared-kernel product
    of the same shape, its error against FP64 on 64 sampled rows, and a fresh
    5-step IterNCGP fit with per-class kernels (j <= 200, R = 100, tolerance
    1e-5).  value = Newton steps/s of that fit."""
    import numpy as np
    import torch

    import datagen
    from oracle import kernels as ok
    from paper_2310_20285_amd import api

    dev = torch.device("cuda:0")
    w = datagen.config2()
    C = w.C
    ls = [1.5 + 0.25 * c for c in range(C)]
    os_ = [0.8 + 0.1 * c for c in range(C)]
    X = torch.tensor(w.X, dtype=torch.float32, device=dev)
    y = torch.tensor(w.y, dtype=torch.int32, device=dev)
    rng = np.random.default_rng(5)
    v = torch.tensor(rng.standard_normal(w.N * C), dtype=torch.float32, device=dev)

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out_pc = torch.empty_like(v)
    out_sh = torch.empty_like(v)
    ms_pc = timed(lambda: api.glm_kernel_matmul(X, X, v, C, w.kernel, ls, os_, "fp32",
                                                out=out_pc))
    ms_sh = timed(lambda: api.glm_kernel_matmul(X, X, v, C, w.kernel, w.lengthscale,
                                                w.outputscale, "fp32", out=out_sh))
    # error against FP64 on 64 sampled rows
    Xh = X.double().cpu().numpy()
    vh = v.double().cpu().numpy().reshape(w.N, C)
    rows = np.sort(rng.choice(w.N, size=64, replace=False))
    ref = np.empty((64, C))
    for c in range(C):
        Kc = ok.kernel_matrix(Xh[rows], Xh, w.kernel, ls[c], os_[c])
        ref[:, c] = Kc @ vh[:, c]
    got = out_pc.double().cpu().numpy().reshape(w.N, C)[rows]
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    # a fresh 5-step fit with per-class kernels
    def make():
        return api.IterNCGP(X, y, C, w.kernel, ls, os_, policy="cg", j_max=200, rank_limit=100,
                            recycle=True, tol_abs=1e-5, tol_rel=1e-5, precision="fp32",
                            residual_mode="recurrence", max_buffer=300)
    mw = make()
    mw.newton_step()
    torch.cuda.synchronize()
    del mw
    m = make()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [m.newton_step() for _ in range(FIT_STEPS)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    evals = w.N * w.N * C               # one kernel evaluation per pair and class
    res = {
        "metric": "IterNCGP Newton steps/s",
        "value": FIT_STEPS / el,
        "unit": "Newton steps/s",
        "n_gpus": 1, "steps": FIT_STEPS, "warmup": 1,
        "ms_per_step": el / FIT_STEPS * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "per-class kernels: gpc N=20000 D=16 C=5 matern52, lengthscales "
                               f"{ls}, outputscales {os_}; IterNCGP-CG j<=200 R=100 tol 1e-5, "
                               f"one fresh fit of {FIT_STEPS} Newton steps"},
        "product": {"per_class_ms": ms_pc, "shared_kernel_ms": ms_sh,
                    "per_class_over_shared": ms_pc / ms_sh,
                    "per_class_geval_s": evals / ms_pc / 1e6,
                    "rel_err_vs_fp64_64_rows": err,
                    "kernel": "symmetric matrix-core kernel, per-class form: the "
                              "distance once per pair, one transform per class, the "
                              "transposed sums on VALU (the shared form: one transform "
                              "per pair, the transposed sums on MFMA)"},
        "iters_per_step": [i["iters"] for i in infos],
    }
    print(json.dumps(res))


def bench_poisson(args):
    """The paper's Poisson regression schedules: N = 100 points on [0, 1], RBF
    prior (lengthscale 0.1, outputscale 5), 100 solver iterations spread over
    5, 10, 20 or 100 Newton steps (j <= 20, 10, 5, 1), recycling without
    compression, outer tolerance 1e-3, 10 runs with re-drawn counts.  Reported
    per schedule: Newton steps taken, device time, RMSE of the posterior mean
    of the log rate against the true log rate.  value = Newton steps/s over all
    runs of all schedules."""
    import numpy as np
    import torch

    import datagen
    from paper_2310_20285_amd import api

    prec = args.precision or "fp64"
    dt = torch.float64 if prec == "fp64" else torch.float32
    dev = torch.device("cuda:0")
    sched = {}
    total_steps, total_t = 0, 0.0
    for jmax, nsteps in ((20, 5), (10, 10), (5, 20), (1, 100)):
        rec = []
        for run in range(10):
            Xn, yn, f = datagen.poisson(seed=run)
            X = torch.tensor(Xn, dtype=dt, device=dev)
            y = torch.tensor(yn, dtype=torch.int32, device=dev)
            m = api.IterNCGP(X, y, 1, "rbf", 0.1, 5.0, likelihood="poisson", policy="cg",
                             j_max=jmax, rank_limit=-1, recycle=True, precision=prec,
                             residual_mode="recurrence", max_buffer=105)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            taken = 0
            for _ in range(nsteps):
                info = m.newton_step()
                taken += 1
                if info["rel_change"] <= 1e-3:
                    break
            t = time.perf_counter() - t0
            mean, _, _ = m.predict(X, probs=False)
            rmse = float(np.sqrt(np.mean((mean.double().cpu().numpy()[:, 0] - f) ** 2)))
            rec.append((taken, t, rmse))
            total_steps += taken
            total_t += t
        a = np.array(rec)
        sched[f"j<={jmax} x {nsteps} steps"] = {
            "steps_taken_median": float(np.median(a[:, 0])),
            "time_ms_median": float(np.median(a[:, 1]) * 1e3),
            "rmse_log_rate_median": float(np.median(a[:, 2])),
            "rmse_log_rate_min": float(a[:, 2].min()), "rmse_log_rate_max": float(a[:, 2].max())}
    res = {
        "metric": "IterNCGP Newton steps/s",
        "value": total_steps / total_t,
        "unit": "Newton steps/s",
        "n_gpus": 1, "steps": total_steps, "warmup": 0,
        "ms_per_step": total_t / total_steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16"}[prec], "data": "synthetic",
        "config": {"workload": "Poisson regression N=100 D=1 rbf l=0.1 os=5; IterNCGP-CG, "
                               "100 iterations over 5/10/20/100 steps, recycling, outer "
                               "tolerance 1e-3, 10 count draws", "precision": prec},
        "schedules": sched,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
