"""Benchmark: DC-GK / DC-LSQR solves per second on one MI355X.

Default workload (the largest single-GPU configuration): hyperspectral-like
deblurring, n1 = n2 = s = 512, n3 = 64, band-dependent Gaussian blur (sigma
from 1.5 to 4 over the bands), spectral Gaussian field, noise level drawn in
[1e-3, 2e-2].  One step = one solve: 40 Golub-Kahan steps (Algorithm 4) with
FP32 vectors and FP32 slice GEMMs on MFMA, the FP64 projected Tikhonov problem
with GCV (Algorithm 5), X = V_k (*) y -- every stage of the hot path, inputs
resident in HBM.

Printed JSON line (rank 0):
  value        solves/s, counted only if the solve's restoration error is
               within 1.05x of a full FP64 oracle solve of the same input,
               run in the same process
  roofline     the kernel kind with the largest total time inside the timed
               solves, timed by start/stop events that each launch records on
               the library's stream; bound by MFMA or HBM by its arithmetic
               intensity
  cpu_baseline the same full oracle solve, timed on the host cores
  mixed_bf16   the same solve with BF16 slice GEMMs (FP32 accumulation), gated
               the same way

Other workloads: --workload colour256 | video256 | video4 | batch64 | paper | longtube |
longsolve | learned512.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload hyper512]
                       [--gemm f32|bf16|f16] [--no-cpu-baseline] [--copy-calib-mib M]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LSQR solves/s at ≤1.05× FP64-oracle error; c-product GB/s & MFMA util"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the fused products at this workload (FP32 GEMMs), from
# two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by a 1 GiB copy read
# in the same runs.  They describe the kernel sources with this digest only.
TRAFFIC_SOURCES = ("paper_2103_11847_amd/csrc/fused.hip", "paper_2103_11847_amd/csrc/mfma.h",
                   "paper_2103_11847_amd/csrc/internal.h")
TRAFFIC = {"digest": "a44b9d1d32ecbf2c", "gemm": "f32",
           "bytes": {"fused_fwd": 6677688, "fused_adj": 6637664}}


# The same for the O(p log p) tube transform at 512 x 512 positions, p = 256, FP32 (bytes per launch).
LONGTUBE_SOURCES = ("paper_2103_11847_amd/csrc/fastdct.hip", "paper_2103_11847_amd/csrc/fastdct.h")
LONGTUBE_TRAFFIC = {"digest": "2b4748b4b2668618", "bytes": 656636507}

# The same for the slice GEMMs and the paired transforms of the 512 x 512 x 64 solve
# (bytes per launch, keyed "gemm type/kernel"), from the counter passes of the hyper512 bench.
HYPER_TRAFFIC_SOURCES = ("paper_2103_11847_amd/csrc/gemm.hip", "paper_2103_11847_amd/csrc/transform.hip",
                         "paper_2103_11847_amd/csrc/mfma.h", "paper_2103_11847_amd/csrc/internal.h")
HYPER_TRAFFIC = {"digest": "50678c7cb80bf0dd",
                 "bytes": {"f32/gemm": 202097938, "f32/tube_pair": 268908161, "bf16/gemm": 134564564, "bf16/tube_pair": 235377510}}


def source_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind, gemm):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != TRAFFIC["digest"] or gemm != TRAFFIC["gemm"]:
        return None
    return TRAFFIC["bytes"].get(kind)
MFMA_PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "f16": 2500.0, "f64": 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 for hyper512, 50 for the other workloads)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default: 3 for hyper512, else 5)")
    ap.add_argument("--gemm", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cprod-reps", type=int, default=200,
                    help="standalone c-product launches timed after the solves (0: none)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run 3 plain device copies of this many MiB (HBM counter calibration)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch64: keep the size-based product paths instead of timing them per shape")
    ap.add_argument("--learned", action="store_true",
                    help="batch64: train the stopping network on the library's own solves of 256 smaller "
                         "problems of the same family, run the batch with the learned stop, and compare "
                         "with plain FP32 single solves")
    ap.add_argument("--lambda-rule", default="gcv", choices=["gcv", "discrepancy", "lcurve"],
                    help="colour256: lambda by GCV (default), by the discrepancy principle at 1.05 x the "
                         "norm of the added noise, or LSQR stopped at the L-curve corner")
    ap.add_argument("--workload", default="hyper512",
                    choices=["hyper512", "colour256", "batch64", "video256", "paper", "longtube", "learned512",
                             "video4", "longsolve"],
                    help="hyper512: one 512x512x64 solve per step (default); colour256: one 256x256x3 "
                         "solve per step; batch64: the uneven 64-instance batch per step (merged launches, "
                         "HIP graph)")
    ap.add_argument("--no-mixed", action="store_true", help="hyper512: skip the BF16-GEMM leg")
    ap.add_argument("--stop-quantile", type=float, default=0.97,
                    help="learned stop: margin added to the predicted step, the quantile of (label - prediction) "
                         "over the training problems")
    ap.add_argument("--mixed-min-n", type=int, default=128,
                    help="batch64 with 16-bit GEMMs: instances with n below this keep FP32 slice GEMMs")
    ap.add_argument("--lambda-gate", type=float, default=1.0,
                    help="learned stop: the predicted lambda is kept when GCV(prediction) <= this x min GCV at the "
                         "predicted step (1.0: the GCV minimiser unless the prediction is as good)")
    ap.add_argument("--train-count", type=int, default=20000,
                    help="learned512: training problems (128x128x64, same family) for the stopping network")
    ap.add_argument("--eval-count", type=int, default=8,
                    help="learned512: 512x512x64 problems solved (each gated on its own FP64 oracle solve)")
    a = ap.parse_args()
    if a.steps is None:
        a.steps = 20 if a.workload in ("hyper512", "longsolve") else 50
    if a.warmup is None:
        a.warmup = 3 if a.workload in ("hyper512", "longsolve") else 5
    return a


def blas_threads():
    try:
        import threadpoolctl
        n = [d.get("num_threads", 0) for d in threadpoolctl.threadpool_info() if d.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()


def oracle_leg(w, C_ref_builder, budget_s, target=None, lcurve=False):
    """FP64 oracle: restoration error on the same input, and timed solves (bounded sample).
    target: lambda by the discrepancy principle at this residual norm (else GCV);
    lcurve: LSQR stopped at the L-curve corner instead."""
    from oracle import krylov, metrics, tikhonov
    from oracle.cprod import Operator, fro
    op = Operator(w["A"])
    Ch = op.apply(w["X_true"])
    C = Ch + w["nu"] * fro(Ch) / fro(w["N0"]) * w["N0"]
    mode = "rect" if target is None else "discrepancy"

    def solve():
        if lcurve:
            g = krylov.gkb(op, C, w["iters"])
            res, nrm = tikhonov.lcurve_points(g.bidiagonal(g.steps), g.beta[0], g.steps)
            k = tikhonov.lcurve_corner(res, nrm)
            out = krylov.dc_lsqr(op, C, k)
            out["lambda"] = float(k)
            return out
        return krylov.dc_gk(op, C, w["iters"], lam=None, gcv_mode=mode, reorth="none", target=target)
    ref = solve()
    err = metrics.relative_error(w["X_true"], ref["X"])
    if budget_s is None:
        return err, ref["lambda"], None, 0, 0.0
    n = 0
    t0 = time.perf_counter()
    while True:
        solve()
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return err, ref["lambda"], n / dt, n, dt


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (--gpus %d requested); how the path would "
              "shard over several GPUs is described, not implemented" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2103_11847_amd as dk
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload in ("hyper512", "video4", "longsolve"):
        return bench_hyper(args)
    if args.workload == "learned512":
        return bench_learned512(args)
    if args.workload == "video256":
        return bench_large(args)
    if args.workload == "paper":
        return bench_paper(args)
    if args.workload == "longtube":
        return bench_longtube(args)
    dev = torch.device("cuda:0")
    w = W.colour_256()
    p, n, s, k = 3, 256, 256, w["iters"]
    gdt = dk.DTYPES[args.gemm]

    ctx = dk.dctk_create(0)
    A64 = torch.from_numpy(w["A"]).to(dev)
    # observation C = M(X_true) + noise at relative level nu, formed with the library's FP64 product
    op64 = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F64, A64, s)
    Xt = torch.from_numpy(w["X_true"]).to(dev)
    Ch = torch.empty_like(Xt)
    dk.dctk_cprod(ctx, op64, 1.0, Xt, 0.0, Ch)
    N0 = torch.from_numpy(w["N0"]).to(dev)
    C64 = Ch + w["nu"] * torch.linalg.norm(Ch) / torch.linalg.norm(N0) * N0
    dk.dctk_op_destroy(op64)

    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, A64, s)
    C = C64.to(torch.float32).contiguous()
    X = torch.empty_like(C)
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, k)
    # lambda by GCV, or by the discrepancy principle at 1.05 x the added noise's norm
    target = None
    if args.lambda_rule == "discrepancy":
        target = 1.05 * float(w["nu"]) * float(torch.linalg.norm(Ch))
        opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 2, -1.0, 0.0, target)
    else:
        opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0, 0.0)

    lcurve = args.lambda_rule == "lcurve"
    k_opt = [None]

    def solve(read=True):
        if lcurve:  # LSQR at the L-curve corner (reads its index back)
            out, k_opt[0] = dk.dctk_lsqr_lcurve_solve(ctx, ws, C, X, opts)
            return out
        return dk.dctk_lsqr_tik_solve(ctx, ws, C, X, opts, info=read)

    for _ in range(args.warmup):
        info = solve()
    torch.cuda.synchronize()
    # timed: the solves are enqueued back to back (no per-solve read-back of the
    # solve info, so the device never waits for the host)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solve(read=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # the same with the info read back after every solve (one host round trip each)
    t0s = time.perf_counter()
    for _ in range(args.steps):
        info = solve()
    torch.cuda.synchronize()
    ms_sync = (time.perf_counter() - t0s) * 1e3 / args.steps

    # independent solves on two streams: two contexts, each with its own operator
    # and workspace, on two torch streams (default priority), solves alternating
    two = None
    if not lcurve:
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        ctx2 = [dk.dctk_create(0, st_) for st_ in streams]
        ops2 = [dk.dctk_op_create(c_, dk.DCTK_TUBE_TH, gdt, A64, s) for c_ in ctx2]
        ws2 = [dk.dctk_krylov_create(c_, o_, dk.DCTK_KRYLOV_GKB, k) for c_, o_ in zip(ctx2, ops2)]
        X2 = [torch.empty_like(C) for _ in range(2)]
        torch.cuda.synchronize()
        for j in range(2):
            dk.dctk_lsqr_tik_solve(ctx2[j], ws2[j], C, X2[j], opts)
        torch.cuda.synchronize()
        t0t = time.perf_counter()
        for i in range(args.steps):
            j = i % 2
            dk.dctk_lsqr_tik_solve(ctx2[j], ws2[j], C, X2[j], opts, info=False)
        torch.cuda.synchronize()
        dt2 = time.perf_counter() - t0t
        same = bool(torch.equal(X2[0], X2[1]))
        two = {"solves_per_s": args.steps / dt2, "ms_per_solve": dt2 * 1e3 / args.steps, "outputs_equal": same,
               "note": "independent solves alternating over two contexts on two streams (the value above is one "
                       "stream)"}
        for j in range(2):
            dk.dctk_krylov_destroy(ws2[j])
            dk.dctk_op_destroy(ops2[j])
            dk.dctk_destroy(ctx2[j])

    # restoration error of the benchmarked solve
    kr = dk.dctk_krylov_read(ctx, ws, k, dk.DCTK_KRYLOV_GKB)
    Xn = X.double().cpu().numpy()
    err_gpu = float(np.linalg.norm((Xn - w["X_true"]).ravel()) / np.linalg.norm(w["X_true"].ravel()))

    # dominant kernel, timed live with HIP events (on the library's stream) around every
    # c-product launch inside the solves
    prof_steps = max(3, min(10, args.steps))
    dk.dctk_profile_begin(ctx)
    for _ in range(prof_steps):
        solve()
    prof = dk.dctk_profile_end(ctx)
    kind = max(("fused_fwd", "fused_adj", "gemm"), key=lambda k_: prof[k_][0])
    k_ms, k_n = prof[kind]
    k_us = k_ms * 1e3 / max(1, k_n)
    flops = 2.0 * n * n * s * p  # the p slice GEMMs of one product (dense-equivalent)
    bg = 4 if args.gemm == "f32" else 2
    N = p * n * s
    # algorithmic bytes of one launch inside a GKB step: A~ once, the input, the epilogue's
    # src (the previous basis vector) and the output -- the Tikhonov steps keep their basis
    # vectors unnormalised, so no normalised copy of the input is written
    nvec_io = {"fused_fwd": 3, "fused_adj": 3, "gemm": 2}[kind]
    kbytes = p * n * n * bg + nvec_io * N * 4
    peak_f = MFMA_PEAK_TFLOPS[args.gemm]
    ridge = peak_f * 1e12 / (HBM_PEAK_GBS * 1e9)
    ai = flops / kbytes
    if ai >= ridge:
        roof = {"bound": "mfma", "achieved": flops / (k_us * 1e-6) / 1e12, "peak": peak_f, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": kbytes / (k_us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(kind, args.gemm)
    roof.update({"kernel": {"fused_fwd": "fused c-product M(X) (transform + p slice MFMA GEMMs + inverse)",
                            "fused_adj": "fused adjoint c-product M*(Y)",
                            "gemm": "slice GEMM batch"}[kind],
                 "avg_us": k_us, "launches": k_n, "flops_per_launch": flops, "bytes_per_launch": kbytes,
                 "arith_intensity": ai,
                 "per_kind_avg_us": {k_: (v[0] * 1e3 / v[1] if v[1] else None) for k_, v in prof.items()}})

    # one c-product, standalone, on the library's stream (the context uses the null stream)
    cprod = None
    if args.cprod_reps > 0:
        Y = torch.empty_like(C)
        for _ in range(5):
            dk.dctk_cprod(ctx, op, 1.0, C, 0.0, Y)
        torch.cuda.synchronize()
        reps = args.cprod_reps
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            dk.dctk_cprod(ctx, op, 1.0, C, 0.0, Y)
        ev1.record()
        torch.cuda.synchronize()
        cprod_us = ev0.elapsed_time(ev1) * 1e3 / reps
        gb = (p * n * n * bg + 2 * N * 4) / 1e9
        cprod = {"us": cprod_us, "GB_per_s": gb / (cprod_us * 1e-6), "hbm_frac": gb / (cprod_us * 1e-6) / HBM_PEAK_GBS,
                 "mfma_frac": flops / (cprod_us * 1e-6) / 1e12 / peak_f, "cprods_per_s": 1e6 / cprod_us}
    if args.copy_calib_mib > 0:
        nel = args.copy_calib_mib * (1 << 20) // 4
        src_b = torch.ones(nel, dtype=torch.float32, device=dev)
        dst_b = torch.empty_like(src_b)
        for _ in range(3):
            dst_b.copy_(src_b)
        torch.cuda.synchronize()
        del src_b, dst_b

    # the oracle's restoration error gates the line whether or not its solves are timed
    cpu = None
    err_oracle, lam_oracle, cps, nsolve, dt = oracle_leg(w, None, None if args.no_cpu_baseline else args.cpu_seconds,
                                                         target, args.lambda_rule == "lcurve")
    if not args.no_cpu_baseline:
        threads = blas_threads()
        cpu = {"value": cps, "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": "%d full FP64 DC-GK solves (40 GKB steps + %s) of the same 256x256x3 workload "
                         "in %.1f s (numpy, BLAS matmul)"
                         % (nsolve, {"gcv": "GCV", "discrepancy": "discrepancy principle",
                                     "lcurve": "L-curve stopping index"}[args.lambda_rule], dt)}
    gate_ok = err_gpu <= 1.05 * err_oracle
    solves_per_s = 1e3 / ms_per_step
    value = solves_per_s if gate_ok else 0.0

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.gemm if args.gemm != "f32" else "f32",
        "data": "synthetic",
        "config": {"workload": "colour deblur 256x256x3, DC-LSQR/DC-GK 40 GKB steps + FP64 %s, one solve per step"
                               % {"gcv": "GCV", "discrepancy": "discrepancy principle",
                                  "lcurve": "L-curve stopping index"}[args.lambda_rule],
                   "lambda_rule": args.lambda_rule,
                   "n1": n, "n2": n, "s": s, "n3": p, "gkb_steps": k, "gemm_dtype": args.gemm,
                   "vector_dtype": "f32", "reorth": "none", "tube": "th"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "restoration": {"relerr_gpu": err_gpu, "relerr_oracle_fp64": err_oracle,
                        "ratio": err_gpu / err_oracle, "gate_1_05": gate_ok,
                        "lambda_gpu": info.lam, "lambda_oracle": None if lcurve else lam_oracle, "iters": info.iters,
                        "jacobi_sweeps": kr["sweeps"] if not lcurve else None,
                        "k_opt_gpu": k_opt[0], "k_opt_oracle": int(lam_oracle) if (lcurve and lam_oracle) else None},
        "cprod": cprod,
        "per_solve_sync": {"solves_per_s": 1e3 / ms_sync, "ms_per_solve": ms_sync,
                           "note": "info read back (host synchronisation) after every solve"},
        "two_streams": two,
    }
    dk.dctk_krylov_destroy(ws)
    dk.dctk_op_destroy(op)
    dk.dctk_destroy(ctx)
    print(json.dumps(line))


# The paper's own runs (Sec. 4, Tables 1 and 3, nu = 1e-3): iteration counts and
# Matlab CPU seconds on an i7-8550U, quoted as context.
PAPER_RUNS = {
    256: {"gmres": (10, 5.21), "gk": (15, 1.62), "lsqr": (14, 1.23)},
    1024: {"gmres": (10, 100.35), "gk": (20, 25.33), "lsqr": (15, 19.45)},
}


def bench_paper(args):
    """The paper-shaped two-sided colour runs at 256^2 x 3 and 1024^2 x 3 with
    synthetic stand-in images: DC-GMRES(10) (10 restart cycles of 10 Arnoldi
    steps, lambda by GCV), DC-GK (mmax steps, GCV) and DC-LSQR (k_opt steps,
    lambda = 0) at the paper's counts, seconds per solve beside the paper's."""
    import torch
    import paper_2103_11847_amd as dk
    import workloads as W
    dev = torch.device("cuda:0")
    gdt = {"f32": dk.DCTK_F32, "bf16": dk.DCTK_BF16, "f16": dk.DCTK_F16}[args.gemm]
    ctx = dk.dctk_create(0)
    table = {}
    runs = max(1, min(args.steps, 5))
    for n in (256, 1024):
        w = W.paper_shaped(n, 1e-3)
        p, _, s = w["X_true"].shape
        A64 = torch.from_numpy(w["A"]).to(dev)
        B64 = torch.from_numpy(w["B"]).to(dev)
        op64 = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F64, A64, s, B64)
        Xt = torch.from_numpy(w["X_true"]).to(dev)
        Ch = torch.empty_like(Xt)
        dk.dctk_cprod(ctx, op64, 1.0, Xt, 0.0, Ch)
        dk.dctk_op_destroy(op64)
        N0 = torch.from_numpy(w["N0"]).to(dev)
        C = (Ch + w["nu"] * torch.linalg.norm(Ch) / torch.linalg.norm(N0) * N0).to(torch.float32).contiguous()
        op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, A64, s, B64)
        X = torch.zeros_like(C)
        row = {}
        for meth in ("gmres", "gk", "lsqr"):
            its, paper_s = PAPER_RUNS[n][meth]
            if meth == "gmres":
                ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_ARNOLDI, 10)
                opts = dk.make_opts(10, dk.DCTK_REORTH_NONE, 0, -1.0, 0.0)

                def solve():
                    X.zero_()
                    return dk.dctk_gmres_tik_solve(ctx, ws, C, X, its, opts)
            else:
                ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, its)
                opts = dk.make_opts(its, dk.DCTK_REORTH_NONE, 0, -1.0 if meth == "gk" else 0.0, 0.0)

                def solve():
                    return dk.dctk_lsqr_tik_solve(ctx, ws, C, X, opts)
            info = solve()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(runs):
                info = solve()
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / runs
            if n == 1024 and meth == "gk":
                # kernel times of the headline row: every transform / GEMM launch of one more solve
                dk.dctk_profile_begin(ctx)
                solve()
                prof_gk = dk.dctk_profile_end(ctx)
            err = float(torch.linalg.norm(X.double() - Xt) / torch.linalg.norm(Xt))
            row[meth] = {"iterations": its, "gpu_s": sec, "relerr": err, "lambda": info.lam,
                         "paper_cpu_s": paper_s, "paper_over_gpu": paper_s / sec}
            dk.dctk_krylov_destroy(ws)
        table["%dx%dx3" % (n, n)] = row
        dk.dctk_op_destroy(op)
    gk = table["1024x1024x3"]["gk"]
    # roofline of the dominant kernel kind of the 1024^2 x 3 DC-GK solve (two-sided:
    # each product is a transform, two slice-GEMM launches, an inverse transform)
    bg = {"f32": 4, "bf16": 2, "f16": 2}[args.gemm]
    n, p = 1024, 3
    kinds = {}
    for kind in ("tube_fwd", "gemm", "tube_inv", "tube_pair"):
        tot, cnt = prof_gk[kind]
        if cnt:
            f, b = kernel_work(kind, p, n, n, n, bg, per_solve=cnt)
            kinds[kind] = roofline_entry(kind, tot * 1e3 / cnt, f, b, args.gemm, None)
            kinds[kind].update({"launches": cnt, "ms_total": tot})
    dom = max(kinds, key=lambda k_: kinds[k_]["ms_total"])
    roof = dict(kinds[dom])
    roof["per_kind"] = kinds
    # the FP64 oracle on every row (the gate), its 1024^2 x 3 DC-GK solve timed
    from oracle import krylov, metrics
    from oracle.cprod import Operator, fro
    gate_all, t_gk = True, None
    for n_, meths in PAPER_RUNS.items():
        w = W.paper_shaped(n_, 1e-3)
        t0 = time.perf_counter()
        orc = Operator(w["A"], w["B"])
        Cn = orc.apply(w["X_true"])
        Cn = Cn + w["nu"] * fro(Cn) / fro(w["N0"]) * w["N0"]
        t_setup = time.perf_counter() - t0
        for meth, (its, _) in meths.items():
            t0 = time.perf_counter()
            if meth == "gmres":
                Xo = krylov.dc_gmres(orc, Cn, np.zeros_like(Cn), 10, its, lam=None)["X"]
            elif meth == "gk":
                Xo = krylov.dc_gk(orc, Cn, its, lam=None)["X"]
            else:
                Xo = krylov.dc_lsqr(orc, Cn, its)["X"]
            dt = time.perf_counter() - t0
            if n_ == 1024 and meth == "gk":
                t_gk = dt + t_setup
            row = table["%dx%dx3" % (n_, n_)][meth]
            row["relerr_oracle_fp64"] = metrics.relative_error(w["X_true"], Xo)
            row["ratio"] = row["relerr"] / row["relerr_oracle_fp64"]
            row["gate_1_05"] = row["ratio"] <= 1.05
            gate_all = gate_all and row["gate_1_05"]
            print("paper: oracle %dx%dx3 %s done (%.1f s)" % (n_, n_, meth, dt), file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": (1.0 / gk["gpu_s"]) if gk["gate_1_05"] else 0.0,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": runs,
        "warmup": 1,
        "ms_per_step": gk["gpu_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.gemm,
        "data": "synthetic",
        "config": {"workload": "paper-shaped two-sided colour deblur 1024x1024x3 (sigma 4, r 6, A_color tube "
                               "(0.8, 0, 0.1), nu 1e-3), DC-GK 20 steps + FP64 GCV, one solve per step",
                   "gemm_dtype": args.gemm, "vector_dtype": "f32"},
        "roofline": roof,
        "cpu_baseline": None if args.no_cpu_baseline else {
            "value": 1.0 / t_gk, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
            "sample": "one full FP64 DC-GK solve (20 steps + GCV, operator set-up and C included) of the same "
                      "1024x1024x3 two-sided problem in %.1f s (numpy, BLAS matmul)" % t_gk},
        "all_rows_within_1_05": gate_all,
        "paper_tables": table,
        "note": "paper_cpu_s: the paper's Matlab seconds on an i7-8550U with its images (Tables 1, 3); "
                "context only, different machine and inputs",
    }
    dk.dctk_destroy(ctx)
    print(json.dumps(line))


def bench_longtube(args):
    """The O(p log p) tube transform on a hyperspectral-shaped cube: 512 x 512
    positions, p = 256 bands, FP32, one step = M (Remark 2.1) applied to every
    tube.  Each element is read and written once (8 bytes per element per
    launch in FP32), so the roofline is HBM.  Also: the four matrices of the
    family, other tube lengths at the same positions, sampled outputs against
    the oracle's dense matrix, and the oracle's dense mode-3 product timed on a
    sample of positions."""
    import torch
    import paper_2103_11847_amd as dk
    from oracle import tube as otube
    dev = torch.device("cuda:0")
    ctx = dk.dctk_create(0)
    p, n = 256, 512
    count = n * n
    gen = torch.Generator(device=dev)
    gen.manual_seed(256)
    x = torch.randn((p, count), device=dev, generator=gen)
    out = torch.empty_like(x)
    TH = dk.DCTK_TUBE_TH

    def avg_seconds(fn, reps):
        fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) * 1e-3 / reps

    def fwd():
        dk.dctk_tube_fast(ctx, TH, dk.DCTK_MAT_L, x, out)

    for _ in range(args.warmup):
        fwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    avg = avg_seconds(fwd, 50)
    bytes_launch = 2 * p * count * 4
    # sampled positions against the oracle's dense M
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(count, 256, replace=False))
    it = torch.from_numpy(idx).to(dev)
    xs = x[:, it].double().cpu().numpy()
    G = otube.transform_matrix(p, "th")
    ref = G @ xs
    got = out[:, it].double().cpu().numpy()
    relerr = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    names = {"M": dk.DCTK_MAT_L, "M_inv": dk.DCTK_MAT_LINV, "M_invT": dk.DCTK_MAT_LINVT, "M_T": dk.DCTK_MAT_LT}
    per_matrix = {}
    for name, which in names.items():
        us = avg_seconds(lambda: dk.dctk_tube_fast(ctx, TH, which, x, out), 30) * 1e6
        per_matrix[name] = {"us": us, "GB_per_s": bytes_launch / (us * 1e-6) / 1e9}
    by_p = {}
    for pl in (16, 64, 1024, 4096):
        xl = torch.randn((pl, count), device=dev, generator=gen)
        ol = torch.empty_like(xl)
        us = avg_seconds(lambda: dk.dctk_tube_fast(ctx, TH, dk.DCTK_MAT_L, xl, ol), 20) * 1e6
        by_p[str(pl)] = {"us": us, "GB_per_s": 2 * pl * count * 4 / (us * 1e-6) / 1e9}
        del xl, ol
    if args.copy_calib_mib > 0:
        # a plain copy of known size, for scaling the HBM counters of a profiled run
        cal = torch.ones(args.copy_calib_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        cal_out = torch.empty_like(cal)
        for _ in range(3):
            cal_out.copy_(cal)
        torch.cuda.synchronize()
        del cal, cal_out
    achieved = bytes_launch / avg / 1e9
    traffic = LONGTUBE_TRAFFIC["bytes"] if source_digest(LONGTUBE_SOURCES) == LONGTUBE_TRAFFIC["digest"] else None
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's dense transform (G @ tubes, numpy/BLAS) over blocks of positions
        xs_all = x[:, :65536].double().cpu().numpy()
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < min(args.cpu_seconds, 15.0):
            otube.mode3(xs_all.reshape(p, 256, 256), G)
            done += 65536
        el = time.perf_counter() - t0
        cpu = {"value": done / count / el, "unit": "transforms/s", "cores": blas_threads(), "kind": "oracle",
               "sample": "%d positions (blocks of 65536 of the 262144) through the oracle's dense FP64 mode-3 "
                         "product in %.1f s, scaled to whole 512x512x256 transforms" % (done, el)}
    # the line counts only while the sampled outputs agree with the oracle's dense M
    # to the FP32 tolerance of the parity tests (1e-6 + 8e-9 p relative 2-norm)
    gate = relerr <= 1e-6 + 8e-9 * p
    line = {
        "metric": "tube transforms/s (M of Remark 2.1 on every tube)",
        "value": (1.0 / sec) if gate else 0.0,
        "unit": "transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "long-tube transform, hyperspectral-shaped 512x512 positions x 256 bands, FP32, "
                               "O(p log p) (FFT-based DCT-II)", "p": p, "positions": count},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "tube_fast_kernel<float>",
                     "avg_us": avg * 1e6, "bytes_per_launch": bytes_launch},
        "cpu_baseline": cpu,
        "sampled_relerr_vs_oracle": relerr,
        "gate": {"tolerance": 1e-6 + 8e-9 * p, "passed": gate},
        "per_matrix": per_matrix,
        "by_p": by_p,
    }
    dk.dctk_destroy(ctx)
    print(json.dumps(line))


def oracle_batch_leg(insts, k, budget_s):
    """FP64 oracle on the batch's instances, smallest first, until budget_s is spent
    (None: every instance): restoration errors and the time taken."""
    from oracle import krylov, metrics
    from oracle.cprod import Operator, fro
    order = sorted(range(len(insts)), key=lambda i: insts[i]["w"]["A"].size * insts[i]["w"]["X_true"].shape[2])
    errs, n, t0 = {}, 0, time.perf_counter()
    for i in order:
        w = insts[i]["w"]
        op = Operator(w["A"])
        Ch = op.apply(w["X_true"])
        C = Ch + w["nu"] * fro(Ch) / fro(w["N0"]) * w["N0"]
        r = krylov.dc_gk(op, C, k, lam=None, gcv_mode="rect", reorth="none")
        errs[i] = metrics.relative_error(w["X_true"], r["X"])
        n += 1
        if n % 8 == 0:
            print("oracle: %d solves done (%.0f s)" % (n, time.perf_counter() - t0), file=sys.stderr, flush=True)
        if budget_s is not None and time.perf_counter() - t0 >= budget_s:
            break
    return errs, n, time.perf_counter() - t0


def bench_batch(args):
    """The uneven 64-instance batch: one step = all 64 DC-GK solves (40 GKB steps + GCV each)."""
    import torch
    import paper_2103_11847_amd as dk
    import workloads as W
    dev = torch.device("cuda:0")
    gdt = dk.DTYPES[args.gemm]
    k = 40
    ctx = dk.dctk_create(0)
    insts = []
    tuned = {}
    flops = 0.0
    for i in range(64):
        w = W.batch_instance(i)
        p, n = w["A"].shape[0], w["A"].shape[1]
        A64 = torch.from_numpy(w["A"]).to(dev)
        op64 = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F64, A64, n)
        Xt = torch.from_numpy(w["X_true"]).to(dev)
        Ch = torch.empty_like(Xt)
        dk.dctk_cprod(ctx, op64, 1.0, Xt, 0.0, Ch)
        dk.dctk_op_destroy(op64)
        N0 = torch.from_numpy(w["N0"]).to(dev)
        C = (Ch + w["nu"] * torch.linalg.norm(Ch) / torch.linalg.norm(N0) * N0).to(torch.float32).contiguous()
        # 16-bit slice GEMMs only where the products are bandwidth-bound (n >= --mixed-min-n);
        # smaller, latency-bound instances gain nothing from them and keep FP32
        gdt_i = gdt if (gdt == dk.DCTK_F32 or n >= args.mixed_min_n) else dk.DCTK_F32
        op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt_i, A64, n)
        if not args.no_autotune:
            key = (p, n, gdt_i)
            if key not in tuned:
                tuned[key] = dk.dctk_op_autotune(ctx, op, 5)
            t = tuned[key]
            dk.dctk_op_set_path(op, 0, t["fwd_path"], t["fwd_tile"])
            dk.dctk_op_set_path(op, 1, t["adj_path"], t["adj_tile"])
        ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, k)
        insts.append({"w": w, "op": op, "ws": ws, "C": C, "X": torch.empty_like(C)})
        flops += (2 * k + 1) * 2.0 * n * n * n * p
        del Xt, Ch, N0
    opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0, 0.0)
    mlp, learned_info = None, None
    plain = None
    if args.learned:
        mlp, learned_info = train_stop_network(ctx, args)
        plain = plain_fp32_loop(ctx, insts, k, opts, args)
    # a loop of single solves of the same form (learned or not)
    def single(it):
        if mlp is not None:
            dk.dctk_lsqr_learned_solve(ctx, it["ws"], mlp, it["C"], it["X"], opts, args.lambda_gate)
        else:
            dk.dctk_lsqr_tik_solve(ctx, it["ws"], it["C"], it["X"], opts)
    for it in insts:
        single(it)
    ref = [it["X"].clone() for it in insts]
    loop_steps = max(1, min(3, args.steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(loop_steps):
        for it in insts:
            single(it)
    torch.cuda.synchronize()
    loop_s = (time.perf_counter() - t0) / loop_steps
    # the batch: merged launches captured in a graph
    b = dk.dctk_batch_create(ctx, [it["ws"] for it in insts], [it["C"] for it in insts],
                             [it["X"] for it in insts], opts, True, mlp=mlp, gate=args.lambda_gate)
    merged, single = dk.dctk_batch_stats(b)
    for _ in range(args.warmup):
        dk.dctk_batch_run(ctx, b)
    dk.dctk_synchronize(ctx)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dk.dctk_batch_run(ctx, b)
    dk.dctk_synchronize(ctx)
    batch_s = (time.perf_counter() - t0) / args.steps
    infos = dk.dctk_batch_info(ctx, b, len(insts))
    k_used = [x.iters for x in infos]
    same = all(torch.equal(it["X"], r) for it, r in zip(insts, ref))
    errs = []
    for it in insts:
        Xn = it["X"].double().cpu().numpy()
        Xt = it["w"]["X_true"]
        errs.append(float(np.linalg.norm((Xn - Xt).ravel()) / np.linalg.norm(Xt.ravel())))
    # every instance is gated on its own full FP64 oracle solve (also without the
    # baseline report); only the instances that pass count in `value`
    oerr, nsolve, dt = oracle_batch_leg(insts, k, None)
    oratios = [errs[i] / oerr[i] for i in range(len(insts))]
    worst = max(oratios)
    passed = [r <= 1.05 for r in oratios]
    cpu = None
    if not args.no_cpu_baseline:
        elems = sum(it["w"]["X_true"].size for it in insts)
        cpu = {"value": nsolve / dt, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
               "sample": "all %d FP64 DC-GK solves (40 GKB steps + GCV) of the batch's instances (%d tensor "
                         "elements in all) in %.1f s" % (nsolve, elems, dt)}
    dk.dctk_batch_destroy(b)
    for it in insts:
        dk.dctk_krylov_destroy(it["ws"])
        dk.dctk_op_destroy(it["op"])
    target = None
    if plain is not None:
        ratios = np.array(errs) / np.array(plain["errs"])
        target = {"plain_fp32_single_solves_per_s": 64.0 / plain["loop_s"],
                  "speedup_vs_plain_fp32_single": plain["loop_s"] / batch_s,
                  "relerr_ratio_vs_plain_fp32": {"median": float(np.median(ratios)),
                                                 "p90": float(np.quantile(ratios, 0.9)),
                                                 "max": float(ratios.max()),
                                                 "frac_within_1_05": float(np.mean(ratios <= 1.05))},
                  "mean_steps": float(np.mean(k_used)), "network": learned_info}
    if mlp is not None:
        dk.dctk_mlp_destroy(mlp)
    dk.dctk_destroy(ctx)
    # the batch must reproduce its single solves; then the gated instances count
    value = (sum(passed) / batch_s) if same else 0.0
    peak = MFMA_PEAK_TFLOPS[args.gemm]
    sizes = collections_count([(it["w"]["A"].shape[1], it["w"]["A"].shape[0]) for it in insts])
    line = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": batch_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.gemm, "data": "synthetic",
        "config": {"workload": "uneven batch of 64 DC-GK solves (n=s in {64..512}, n3 in {3,8,31}, %s "
                               "+ FP64 GCV each), one batch per step, merged launches in a HIP graph"
                               % ("learned stop after 8 of up to 40 GKB steps" if args.learned else "40 GKB steps"),
                   "instances": 64, "gkb_steps": k, "gemm_dtype": args.gemm, "sizes_n_n3": sizes,
                   "mixed_min_n": args.mixed_min_n,
                   "autotuned_paths": {"%dx%d/%d" % (kk[1], kk[0], kk[2]): v for kk, v in tuned.items()}},
        "roofline": {"bound": "mfma", "achieved": flops / batch_s / 1e12, "peak": peak, "unit": "TFLOP/s",
                     "frac": flops / batch_s / 1e12 / peak, "traffic": None,
                     "kernel": "whole batch step (slice-GEMM flops of all 81 products per instance)"},
        "cpu_baseline": cpu,
        "batch": {"loop_of_single_solves_per_s": 64.0 / loop_s, "speedup_vs_loop": loop_s / batch_s,
                  "launches_merged": merged, "launches_single": single, "bitwise_equal_to_single": same,
                  "worst_relerr_ratio_vs_oracle": worst, "instances_passing_1_05": int(sum(passed)),
                  "relerr_ratio_vs_oracle": oratios, "median_relerr": float(np.median(errs)),
                  "lambda_range": [min(x.lam for x in infos), max(x.lam for x in infos)]},
        "target_form": target,
    }
    print(json.dumps(line))


def train_stop_network(ctx, args):
    """The stopping network, trained on the library's own FP32 solves of 1024 smaller
    problems of the batch's family (labels from their restoration errors)."""
    import paper_2103_11847_amd as dk
    from paper_2103_11847_amd import learned_stop as ls
    import workloads as W
    t0 = time.perf_counter()
    data = ls.make_dataset(ctx, (W.batch_train_instance(i) for i in range(1024)),
                           progress=lambda i: print("batch64: labelled %d training problems (%.0f s)"
                                                    % (i, time.perf_counter() - t0), file=sys.stderr, flush=True))
    t_data = time.perf_counter() - t0
    T, scaling = ls.targets(data)
    m = dk.dctk_mlp_create(ctx, 5)
    dk.dctk_mlp_set_scaling(m, *scaling)
    t0 = time.perf_counter()
    curve = ls.train(ctx, m, data["F"], T, steps=2000)
    t_train = time.perf_counter() - t0
    off = ls.calibrate_offset(ctx, m, data["F"], data["k"], scaling, quantile=args.stop_quantile)
    return m, {"train_problems": int(data["F"].shape[0]), "label_seconds": t_data, "train_seconds": t_train,
               "loss_first_last": [curve[0][1], curve[-1][1]], "stop_offset": off,
               "label_k_mean": float(data["k"].mean())}


def plain_fp32_loop(ctx, insts, k, opts, args):
    """Plain FP32 GPU LSQR (DC-GK, 40 steps, GCV), one solve after another: time and errors."""
    import torch
    import paper_2103_11847_amd as dk
    made = []
    for it in insts:
        w = it["w"]
        op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F32, torch.from_numpy(w["A"]).to("cuda:0"),
                               w["A"].shape[1])
        made.append((op, dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, k)))
    X = [torch.empty_like(it["C"]) for it in insts]
    for (op, ws), it, x in zip(made, insts, X):
        dk.dctk_lsqr_tik_solve(ctx, ws, it["C"], x, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (op, ws), it, x in zip(made, insts, X):
        dk.dctk_lsqr_tik_solve(ctx, ws, it["C"], x, opts)
    torch.cuda.synchronize()
    loop_s = time.perf_counter() - t0
    errs = []
    for it, x in zip(insts, X):
        Xt = it["w"]["X_true"]
        errs.append(float(np.linalg.norm((x.double().cpu().numpy() - Xt).ravel()) / np.linalg.norm(Xt.ravel())))
    for op, ws in made:
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)
    return {"loop_s": loop_s, "errs": errs}


# Algorithmic work per launch of the three kernels of a one-sided product inside a
# GKB step (N = p n s elements per Krylov tensor, b_g bytes per GEMM element):
#   tube_fwd  reads the unnormalised vector, writes its normalised copy (V_j or
#             U_{j+1}) and the transformed tubes in the GEMM type: N (8 + b_g) bytes,
#             2 p N flops
#   gemm      reads A~ (p n1 n2 b_g) and the transformed tubes (N b_g), writes the
#             FP32 slice products (4 N): 2 n1 n2 s p flops
#   tube_inv  reads the slice products and the epilogue's src, writes the output:
#             12 N bytes, 2 p N flops
def kernel_work(kind, p, n1, n2, s, bg, fast=False, per_solve=None):
    """(flops, algorithmic bytes) of one launch, averaged over a DC-GK solve's
    launches of that kind (`per_solve` of them).  Transforms: 2p flops per
    element as a dense p x p product, about 5 log2(p) with the O(p log p)
    transform of long tubes (one complex FFT of length p per tube pair)."""
    N = p * n2 * s
    tf = 5.0 * math.log2(p) * N if fast else 2.0 * p * N
    if kind == "gemm":
        return 2.0 * n1 * n2 * s * p, p * n1 * n2 * bg + N * (bg + 4)
    if kind == "tube_fwd":
        # input read, X~ written in the GEMM type (the Tikhonov steps write no
        # normalised copy); the forward transform of the initial product M*(C)
        # also writes U_1 (FP32), once per solve
        return tf, N * (4 + bg) + (4.0 * N / per_solve if per_solve else 0.0)
    if kind == "tube_inv":
        # product rows read, output written; every inverse but that of M*(C)
        # (one per solve) also reads its src
        return tf, 8.0 * N + (4.0 * N * (per_solve - 1) / per_solve if per_solve else 4.0 * N)
    if kind == "tube_pair":
        # the slice products and src read, the new basis vector written, and the
        # next product's transformed input written in the GEMM type; two transforms
        return 2.0 * tf, N * (12 + bg)
    raise ValueError(kind)


def roofline_entry(kind, avg_us, flops, byts, gemm, traffic=None):
    """Bound by arithmetic intensity against the ridge of the kernel's arithmetic:
    the slice GEMM against its MFMA type, the transforms against FP32."""
    peak_f = MFMA_PEAK_TFLOPS[gemm if kind == "gemm" else "f32"]
    ai = flops / byts
    if ai >= peak_f * 1e12 / (HBM_PEAK_GBS * 1e9):
        r = {"bound": "mfma", "achieved": flops / (avg_us * 1e-6) / 1e12, "peak": peak_f, "unit": "TFLOP/s"}
    else:
        r = {"bound": "hbm", "achieved": byts / (avg_us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = traffic
    r.update({"kernel": kind, "avg_us": avg_us, "flops_per_launch": flops, "bytes_per_launch": byts,
              "arith_intensity": ai})
    return r


def hyper_traffic(kind, gemm):
    """HBM bytes per launch from the rocprofv3 counter passes, while the sources match."""
    if source_digest(HYPER_TRAFFIC_SOURCES) != HYPER_TRAFFIC["digest"]:
        return None
    return HYPER_TRAFFIC["bytes"].get("%s/%s" % (gemm, kind))


def bench_hyper(args):
    """hyper512: one DC-GK solve (40 GKB steps, FP64 GCV) of the 512 x 512 x 64
    hyperspectral-like problem per step, gated on a full FP64 oracle solve.
    video4: the same for the order-4 colour video (128 x 128 x 3 colours x 16
    frames, an order-4 operator: 48 flattened tube slices)."""
    import torch
    import paper_2103_11847_amd as dk
    import workloads as W
    dev = torch.device("cuda:0")
    order4 = args.workload == "video4"
    longsolve = args.workload == "longsolve"
    if order4:
        w = W.colour_video(0)
    elif longsolve:
        w = W.hyperspectral(0, n=256, p=256)
    else:
        w = W.hyperspectral(0)
    shape_name = "128x128x3x16" if order4 else ("256x256x256" if longsolve else "512x512x64")
    n, s = w["X_true"].shape[-2:]
    p = int(np.prod(w["X_true"].shape[:-2]))
    k = w["iters"]
    ctx = dk.dctk_create(0)
    A64 = torch.from_numpy(w["A"]).to(dev)

    def make_op(gdt):
        if order4:
            return dk.dctk_op_create_nd(ctx, dk.DCTK_TUBE_TH, gdt, A64, s)
        return dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, A64, s)
    # C = M(X_true) + noise at relative level nu, formed with the library's FP64 product
    op64 = make_op(dk.DCTK_F64)
    Xt = torch.from_numpy(w["X_true"]).to(dev)
    Ch = torch.empty_like(Xt)
    dk.dctk_cprod(ctx, op64, 1.0, Xt, 0.0, Ch)
    dk.dctk_op_destroy(op64)
    N0 = torch.from_numpy(w["N0"]).to(dev)
    C = (Ch + w["nu"] * torch.linalg.norm(Ch) / torch.linalg.norm(N0) * N0).to(torch.float32).contiguous()
    del Ch, N0
    opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0, 0.0)
    nrm_t = float(torch.linalg.norm(Xt))

    def run(gemm, steps, warmup):
        """Timed region: `steps` solves enqueued back to back (no read-back between
        them).  Then the same number of solves with every transform / GEMM launch
        recording start and stop events on the library's stream (kernel times)."""
        op = make_op(dk.DTYPES[gemm])
        ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, k)
        X = torch.empty_like(C)
        for _ in range(warmup):
            dk.dctk_lsqr_tik_solve(ctx, ws, C, X, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            dk.dctk_lsqr_tik_solve(ctx, ws, C, X, opts, info=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        dk.dctk_profile_begin(ctx)
        t0 = time.perf_counter()
        for _ in range(steps):
            dk.dctk_lsqr_tik_solve(ctx, ws, C, X, opts, info=False)
        torch.cuda.synchronize()
        ms_prof = (time.perf_counter() - t0) * 1e3 / steps
        prof = dk.dctk_profile_end(ctx)
        info = dk.dctk_lsqr_tik_solve(ctx, ws, C, X, opts)
        err = float(torch.linalg.norm(X.double() - Xt)) / nrm_t
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)
        return ms, ms_prof, prof, err, info

    gemm = args.gemm
    ms, ms_prof, prof, err_gpu, info = run(gemm, args.steps, args.warmup)
    bg = {"f32": 4, "bf16": 2, "f16": 2}[gemm]
    kinds = {}
    for kind in ("tube_fwd", "gemm", "tube_inv", "tube_pair"):
        tot, cnt = prof[kind]
        if cnt:
            f, b = kernel_work(kind, p, n, n, s, bg, fast=longsolve, per_solve=cnt / args.steps)
            kinds[kind] = roofline_entry(kind, tot * 1e3 / cnt, f, b, gemm,
                                         None if (order4 or longsolve) else hyper_traffic(kind, gemm))
            kinds[kind].update({"launches": cnt, "ms_total": tot})
    dom = max(kinds, key=lambda k_: kinds[k_]["ms_total"])
    roof = dict(kinds[dom])
    how = "O(p log p)" if longsolve else "MFMA"
    roof["kernel"] = {"gemm": "slice GEMM batch (p MFMA GEMMs of n1 x n2 by n2 x s)",
                      "tube_fwd": "forward tube transform (%s, with the input scale)" % how,
                      "tube_inv": "inverse tube transform (%s, with the epilogue)" % how,
                      "tube_pair": "inverse tube transform with the epilogue paired with the next product's "
                                   "forward transform (MFMA)"}[dom]
    roof["per_kind"] = kinds

    mixed = None
    if not args.no_mixed and gemm == "f32":
        ms_b, _, prof_b, err_b, info_b = run("bf16", args.steps, 2)
        kb = {}
        for kind in ("tube_fwd", "gemm", "tube_inv", "tube_pair"):
            tot, cnt = prof_b[kind]
            if cnt:
                f, b = kernel_work(kind, p, n, n, s, 2, fast=longsolve, per_solve=cnt / args.steps)
                kb[kind] = roofline_entry(kind, tot * 1e3 / cnt, f, b, "bf16",
                                          None if (order4 or longsolve) else hyper_traffic(kind, "bf16"))
                kb[kind].update({"launches": cnt, "ms_total": tot})
        mixed = {"solves_per_s": 1e3 / ms_b, "ms_per_step": ms_b, "relerr_gpu": err_b, "lambda": info_b.lam,
                 "per_kind": kb}

    if args.copy_calib_mib > 0:
        # plain device copies of known size, for scaling the HBM counters of a profiled run
        cal = torch.ones(args.copy_calib_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        cal_out = torch.empty_like(cal)
        for _ in range(3):
            cal_out.copy_(cal)
        torch.cuda.synchronize()
        del cal, cal_out
    # what a plain device copy attains on this GPU (1 read + 1 write stream, 256 MiB
    # buffers taken in turn so the 256 MB last-level cache cannot serve them): context
    # for the transforms' HBM fraction, whose roofline stays the published peak
    bufs = [torch.ones(64 << 20, dtype=torch.float32, device=dev) for _ in range(4)]
    for i in range(4):
        bufs[(i + 1) % 4].copy_(bufs[i])
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for i in range(20):
        bufs[(i + 1) % 4].copy_(bufs[i % 4])
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 20 * 2 * (256 << 20) / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del bufs

    # the FP64 oracle: one full solve of the same problem (its own C), timed
    from oracle import krylov, metrics
    from oracle.cprod import Operator, fro
    from oracle.ordern import OperatorND
    t0 = time.perf_counter()
    orc = OperatorND(w["A"]) if order4 else Operator(w["A"])
    Cn = orc.apply(w["X_true"])
    Cn = Cn + w["nu"] * fro(Cn) / fro(w["N0"]) * w["N0"]
    ref = krylov.dc_gk(orc, Cn, k, lam=None, gcv_mode="rect", reorth="none")
    dt = time.perf_counter() - t0
    err_oracle = metrics.relative_error(w["X_true"], ref["X"])
    cpu = None
    if not args.no_cpu_baseline:
        cpu = {"value": 1.0 / dt, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
               "sample": "one full FP64 DC-GK solve of the same %s problem (operator set-up, C, 40 GKB "
                         "steps, GCV, combine) in %.1f s (numpy, BLAS matmul)" % (shape_name, dt)}
    gate = err_gpu <= 1.05 * err_oracle
    if mixed is not None:
        mixed["ratio_vs_oracle"] = mixed["relerr_gpu"] / err_oracle
        mixed["gate_1_05"] = mixed["relerr_gpu"] <= 1.05 * err_oracle
        mixed["value"] = mixed["solves_per_s"] if mixed["gate_1_05"] else 0.0
        mixed["speedup_vs_f32"] = ms / ms_b
    dk.dctk_destroy(ctx)
    line = {
        "metric": METRIC, "value": (1e3 / ms) if gate else 0.0, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": gemm, "data": "synthetic",
        "config": {"workload": ("order-4 colour video deblur 128x128 x 3 colours x 16 frames (colour tube "
                                "(0.7, 0.15, 0.15) on mode 3, temporal half-kernel on mode 4, Gaussian blur "
                                "sigma 2), DC-GK 40 GKB steps + FP64 GCV, one solve per step" if order4 else
                                "hyperspectral-like deblur %s, band-dependent blur sigma 1.5-4, "
                                "DC-GK 40 GKB steps + FP64 GCV, one solve per step%s"
                                % (shape_name, ", O(p log p) tube transforms" if longsolve else "")),
                   "n1": n, "n2": n, "s": s, "n3": p, "tube_dims": list(reversed(w["X_true"].shape[:-2])),
                   "gkb_steps": k, "gemm_dtype": gemm,
                   "vector_dtype": "f32", "reorth": "none", "tube": "th", "nu": w["nu"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "restoration": {"relerr_gpu": err_gpu, "relerr_oracle_fp64": err_oracle, "ratio": err_gpu / err_oracle,
                        "gate_1_05": gate, "lambda_gpu": info.lam, "lambda_oracle": ref["lambda"],
                        "iters": info.iters},
        "profiled_pass": {"ms_per_step": ms_prof,
                          "note": "the kernel times come from a second pass of the same number of solves in "
                                  "which every launch records start/stop events"},
        "mixed_bf16": mixed,
        "device_copy_GB_per_s": copy_gbs,
    }
    print(json.dumps(line))



def bench_learned512(args):
    """The target form on the 512 x 512 x 64 hyperspectral workload: the
    stopping network trained on the library's own FP32 solves of --train-count
    problems of the same family at 128 x 128 x 64; then --eval-count 512 x 512
    x 64 problems (own fields, noise levels) solved (a) as plain FP32 DC-GK
    single solves (40 GKB steps + GCV) and (b) in the target form: BF16 slice
    GEMMs, the learned stop after 8 steps with the GCV gate, all instances in
    one batch (merged launches, HIP graph).  Every instance of both forms is
    gated on a full FP64 oracle solve of the same problem; `value` counts only
    the target-form solves that pass (within 1.05x of the oracle's error)."""
    import torch
    import paper_2103_11847_amd as dk
    from paper_2103_11847_amd import learned_stop as ls
    import workloads as W
    from oracle import krylov, metrics
    from oracle.cprod import Operator, fro
    dev = torch.device("cuda:0")
    k = 40
    ctx = dk.dctk_create(0)
    # 1. training data from the library's own solves, and training
    t0 = time.perf_counter()
    ntrain = args.train_count
    def note(msg):
        print("learned512: %s (%.0f s)" % (msg, time.perf_counter() - t0), file=sys.stderr, flush=True)
    data = ls.make_family_dataset(ctx, lambda i: W.hyper_family_instance(i, 128), ntrain,
                                  W.hyper_family_operator(128), 128, k_max=k,
                                  progress=lambda i: note("labelled %d problems" % i))
    t_label = time.perf_counter() - t0
    T, scaling = ls.targets(data)
    mlp = dk.dctk_mlp_create(ctx, 21)
    dk.dctk_mlp_set_scaling(mlp, *scaling)
    t0 = time.perf_counter()
    curve = ls.train(ctx, mlp, data["F"], T, steps=3000)
    t_train = time.perf_counter() - t0
    off = ls.calibrate_offset(ctx, mlp, data["F"], data["k"], scaling, quantile=args.stop_quantile)
    # 2. the 512 x 512 x 64 problems
    insts = []
    for i in range(args.eval_count):
        w = W.hyperspectral(i)
        A64 = torch.from_numpy(w["A"]).to(dev)
        op64 = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F64, A64, w["X_true"].shape[2])
        Xt = torch.from_numpy(w["X_true"]).to(dev)
        Ch = torch.empty_like(Xt)
        dk.dctk_cprod(ctx, op64, 1.0, Xt, 0.0, Ch)
        dk.dctk_op_destroy(op64)
        N0 = torch.from_numpy(w["N0"]).to(dev)
        C = (Ch + w["nu"] * torch.linalg.norm(Ch) / torch.linalg.norm(N0) * N0).to(torch.float32).contiguous()
        del Ch, N0
        insts.append({"w": w, "A64": A64, "C": C, "Xt": Xt.to(torch.float32), "nx": float(torch.linalg.norm(Xt))})
        del Xt
    opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0, 0.0)
    s = insts[0]["w"]["X_true"].shape[2]
    # (a) plain FP32 single solves, one after another
    op32 = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F32, insts[0]["A64"], s)
    ws32 = dk.dctk_krylov_create(ctx, op32, dk.DCTK_KRYLOV_GKB, k)
    X = torch.empty_like(insts[0]["C"])
    dk.dctk_lsqr_tik_solve(ctx, ws32, insts[0]["C"], X, opts)
    torch.cuda.synchronize()
    err_plain, t_plain = [], 0.0
    for it in insts:
        t0 = time.perf_counter()
        dk.dctk_lsqr_tik_solve(ctx, ws32, it["C"], X, opts)
        t_plain += time.perf_counter() - t0
        err_plain.append(float(torch.linalg.norm(X - it["Xt"])) / it["nx"])
    dk.dctk_krylov_destroy(ws32)
    dk.dctk_op_destroy(op32)
    del X
    # (b) the target form: BF16 GEMMs + learned stop, all instances in one batch
    made = []
    for it in insts:
        op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_BF16, it["A64"], s)
        ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_GKB, k)
        made.append((op, ws, torch.empty_like(it["C"])))
    b = dk.dctk_batch_create(ctx, [m[1] for m in made], [it["C"] for it in insts], [m[2] for m in made], opts,
                             True, mlp=mlp, gate=args.lambda_gate)
    for _ in range(max(1, args.warmup)):
        dk.dctk_batch_run(ctx, b)
    dk.dctk_synchronize(ctx)
    reps = max(1, min(args.steps, 10))
    t0 = time.perf_counter()
    for _ in range(reps):
        dk.dctk_batch_run(ctx, b)
    dk.dctk_synchronize(ctx)
    t_batch = (time.perf_counter() - t0) / reps
    infos = dk.dctk_batch_info(ctx, b, len(made))
    k_lim, acc = dk.dctk_batch_learned(ctx, b, len(made))
    err_target = [float(torch.linalg.norm(m[2] - it["Xt"])) / it["nx"] for m, it in zip(made, insts)]
    # kernel times of the target form: one learned single solve per instance, profiled
    dk.dctk_profile_begin(ctx)
    for m, it in zip(made, insts):
        dk.dctk_lsqr_learned_solve(ctx, m[1], mlp, it["C"], m[2], opts, args.lambda_gate)
    prof = dk.dctk_profile_end(ctx)
    dk.dctk_batch_destroy(b)
    for op, ws, _ in made:
        dk.dctk_krylov_destroy(ws)
        dk.dctk_op_destroy(op)
    dk.dctk_mlp_destroy(mlp)
    p, n = insts[0]["w"]["X_true"].shape[:2]
    kinds = {}
    for kind in ("tube_fwd", "gemm", "tube_inv", "tube_pair"):
        tot, cnt = prof[kind]
        if cnt:
            f, byt = kernel_work(kind, p, n, n, s, 2, per_solve=cnt / len(made))
            kinds[kind] = roofline_entry(kind, tot * 1e3 / cnt, f, byt, "bf16", hyper_traffic(kind, "bf16"))
            kinds[kind].update({"launches": cnt, "ms_total": tot})
    dom = max(kinds, key=lambda k_: kinds[k_]["ms_total"])
    roof = dict(kinds[dom])
    roof["per_kind"] = kinds
    # 3. the FP64 oracle on every problem (the gate), timed
    err_oracle, t_oracle = [], 0.0
    for it in insts:
        w = it["w"]
        t0 = time.perf_counter()
        orc = Operator(w["A"])
        Cn = orc.apply(w["X_true"])
        Cn = Cn + w["nu"] * fro(Cn) / fro(w["N0"]) * w["N0"]
        ref = krylov.dc_gk(orc, Cn, k, lam=None, gcv_mode="rect", reorth="none")
        t_oracle += time.perf_counter() - t0
        err_oracle.append(metrics.relative_error(w["X_true"], ref["X"]))
        del orc, Cn, ref
        print("learned512: oracle solve %d of %d done" % (len(err_oracle), len(insts)), file=sys.stderr, flush=True)
    ratio_t = [e / o for e, o in zip(err_target, err_oracle)]
    ratio_p = [e / o for e, o in zip(err_plain, err_oracle)]
    passed = [r <= 1.05 for r in ratio_t]
    E = len(insts)
    dk.dctk_destroy(ctx)
    line = {
        "metric": METRIC, "value": sum(passed) / t_batch, "unit": "solves/s", "n_gpus": 1, "steps": reps,
        "warmup": max(1, args.warmup), "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "target form on hyperspectral-like 512x512x64 (band-dependent blur sigma 1.5-4): "
                               "%d problems per step in one batch, BF16 slice GEMMs, learned stop after 8 of up "
                               "to 40 GKB steps + FP64 GCV gate" % E,
                   "n1": n, "n2": n, "s": s, "n3": p, "instances": E, "gemm_dtype": "bf16", "vector_dtype": "f32"},
        "roofline": roof,
        "cpu_baseline": None if args.no_cpu_baseline else {
            "value": E / t_oracle, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
            "sample": "%d full FP64 DC-GK solves (40 GKB steps + GCV) of the evaluated 512x512x64 problems in "
                      "%.1f s (numpy, BLAS matmul)" % (E, t_oracle)},
        "target_form": {
            "solves_per_s": E / t_batch, "gated_solves_per_s": sum(passed) / t_batch,
            "plain_fp32_single_solves_per_s": E / t_plain, "speedup_vs_plain_fp32": t_plain / t_batch,
            "relerr_ratio_vs_oracle": {"target": ratio_t, "plain_fp32": ratio_p, "max_target": max(ratio_t)},
            "instances_passing_1_05": int(sum(passed)), "steps_used": [x.iters for x in infos],
            "learned_step_limit": k_lim, "lambda_accepted": acc},
        "network": {"train_problems": int(data["F"].shape[0]), "train_size": "128x128x64",
                    "label_seconds": t_label, "train_seconds": t_train,
                    "loss_first_last": [curve[0][1], curve[-1][1]], "stop_offset": off,
                    "label_k_mean": float(data["k"].mean()), "label_k_range": [float(data["k"].min()),
                                                                                float(data["k"].max())]},
    }
    print(json.dumps(line))


def bench_large(args):
    """video256: two-sided 256x256x32 DC-GMRES (40 Arnoldi steps, GCV), one solve per
    step; the dominant kernel is timed live."""
    import torch
    import paper_2103_11847_amd as dk
    import workloads as W
    dev = torch.device("cuda:0")
    gdt = dk.DTYPES[args.gemm]
    video = args.workload == "video256"
    w = W.video_256()
    p, n, s = w["X_true"].shape
    k = 40
    ctx = dk.dctk_create(0)
    A64 = torch.from_numpy(w["A"]).to(dev)
    B64 = torch.from_numpy(w["B"]).to(dev) if video else None
    op64 = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, dk.DCTK_F64, A64, s, B64)
    Xt = torch.from_numpy(w["X_true"]).to(dev)
    Ch = torch.empty_like(Xt)
    dk.dctk_cprod(ctx, op64, 1.0, Xt, 0.0, Ch)
    dk.dctk_op_destroy(op64)
    N0 = torch.from_numpy(w["N0"]).to(dev)
    C = (Ch + w["nu"] * torch.linalg.norm(Ch) / torch.linalg.norm(N0) * N0).to(torch.float32).contiguous()
    del Ch, N0
    op = dk.dctk_op_create(ctx, dk.DCTK_TUBE_TH, gdt, A64, s, B64)
    tuned = None if args.no_autotune else dk.dctk_op_autotune(ctx, op, 3)
    ws = dk.dctk_krylov_create(ctx, op, dk.DCTK_KRYLOV_ARNOLDI if video else dk.DCTK_KRYLOV_GKB, k)
    X = torch.zeros_like(C)
    opts = dk.make_opts(k, dk.DCTK_REORTH_NONE, 0, -1.0, 0.0)

    def solve(read_info=True):
        if video:
            X.zero_()
            return dk.dctk_gmres_tik_solve(ctx, ws, C, X, 1, opts)
        return dk.dctk_lsqr_tik_solve(ctx, ws, C, X, opts, info=read_info)
    for _ in range(args.warmup):
        info = solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solve(read_info=False)  # DC-GK: enqueued back to back; DC-GMRES reads its info
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    err = float(torch.linalg.norm(X.double() - Xt) / torch.linalg.norm(Xt))
    dk.dctk_profile_begin(ctx)
    solve()
    prof = dk.dctk_profile_end(ctx)
    kind = max(prof, key=lambda k_: prof[k_][0])
    k_ms, k_n = prof[kind]
    k_us = k_ms * 1e3 / max(1, k_n)
    bg = {"f32": 4, "bf16": 2, "f16": 2}[args.gemm]
    N = p * n * s
    if kind in ("gemm", "fused_fwd", "fused_adj"):
        flops = 2.0 * n * n * s * p * (2 if video else 1)
        byts = p * n * n * bg + (p * s * s * bg if video else 0) + N * (bg + 4 if kind == "gemm" else 8)
    else:  # tube transform: read and write p x n x s, 2p flops per element
        flops = 2.0 * p * N
        byts = N * (4 + (bg if kind == "tube_fwd" else 4))
    peak_f = MFMA_PEAK_TFLOPS[args.gemm]
    if kind.startswith("tube"):
        peak_f = MFMA_PEAK_TFLOPS["f32"]   # vector FP32 arithmetic
    ai = flops / byts
    if ai >= peak_f * 1e12 / (HBM_PEAK_GBS * 1e9):
        roof = {"bound": "mfma" if not kind.startswith("tube") else "alu", "achieved": flops / (k_us * 1e-6) / 1e12,
                "peak": peak_f, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": byts / (k_us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof.update({"traffic": None, "kernel": kind, "avg_us": k_us, "launches": k_n, "flops_per_launch": flops,
                 "bytes_per_launch": byts, "arith_intensity": ai,
                 "per_kind_avg_us": {k_: (v[0] * 1e3 / v[1] if v[1] else None) for k_, v in prof.items()}})
    # the FP64 oracle: one full solve of the same problem (its own C), timed; the gate
    from oracle import krylov, metrics
    from oracle.cprod import Operator, fro
    t0 = time.perf_counter()
    orc = Operator(w["A"], w["B"])
    Cn = orc.apply(w["X_true"])
    Cn = Cn + w["nu"] * fro(Cn) / fro(w["N0"]) * w["N0"]
    ref = krylov.dc_gmres(orc, Cn, np.zeros_like(Cn), k, 1, lam=None)
    dt = time.perf_counter() - t0
    err_oracle = metrics.relative_error(w["X_true"], ref["X"])
    gate = err <= 1.05 * err_oracle
    cpu = None
    if not args.no_cpu_baseline:
        cpu = {"value": 1.0 / dt, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
               "sample": "one full FP64 DC-GMRES solve (40 Arnoldi steps + GCV, operator set-up and C included) "
                         "of the same 256x256x32 two-sided problem in %.1f s (numpy, BLAS matmul)" % dt}
    dk.dctk_krylov_destroy(ws)
    dk.dctk_op_destroy(op)
    dk.dctk_destroy(ctx)
    line = {
        "metric": METRIC, "value": (1e3 / ms) if gate else 0.0, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.gemm, "data": "synthetic",
        "config": {"workload": ("video deblur 256x256x32 two-sided A*X*B, DC-GMRES 40 Arnoldi steps + FP64 GCV"
                                if video else
                                "hyperspectral-like 512x512x64 band-dependent blur, DC-GK 40 GKB steps + FP64 GCV"),
                   "n1": n, "n2": n, "s": s, "n3": p, "krylov_steps": k, "gemm_dtype": args.gemm,
                   "product_paths": tuned},
        "roofline": roof, "cpu_baseline": cpu,
        "restoration": {"relerr_gpu": err, "relerr_oracle_fp64": err_oracle, "ratio": err / err_oracle,
                        "gate_1_05": gate, "lambda": info.lam, "lambda_oracle": ref["lambdas"], "iters": info.iters},
    }
    print(json.dumps(line))


def collections_count(items):
    out = {}
    for n, p in items:
        key = "%dx%d" % (n, p)
        out[key] = out.get(key, 0) + 1
    return out


if __name__ == "__main__":
    main()
