#!/usr/bin/env python3
"""Throughput of the phenotype-panel association scan on one MI355X.

One step = the whole hot path over one synthetic cohort: covariate QR
(tgw_fit_covariates), panel preparation (tgw_prepare_phenotypes), plan and
the scan of every marker (tgw_scan: integer marker statistics, Q^T g,
matrix-core contraction with the fused r/beta/SE/t/-log10 p epilogue and the
FP64 tail), with genotypes, covariates and phenotypes already resident in
HBM.  value = markers x phenotypes / step time.

Prints one JSON line.  Default workload: N=23,000 samples, M=1,000,000
markers, P=2,048 phenotypes, K=10 covariates, split-BF16 precision form; the
plain FP32 scan of the same cohort is timed beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "marker×phenotype tests/s, 1 MI355X: FP8/BF16-split vs FP32 at |Δr|≤1e-5"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PAPER_CONTEXT = {
    "paper_a100_tests_per_s_P2048": 1.94e7,
    "paper_a100_tests_per_s_P20480": 1.65e8,
    "fastgwa_epyc7763_tests_per_s": 8.9e4,
    "note": "paper figures are end-to-end on 8.9M markers x ~23k samples on other hardware; context only",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2604_21095_amd", "csrc", "tgw_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, precision: str):
    """HBM bytes per main-kernel launch measured with rocprofv3 counters, if the
    kernel source has not changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_gemm_{precision}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(spec, n_markers: int):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np

    import oracle
    from synth import geno_codes_np, panel_inputs

    C, Y = panel_inputs(spec)
    codes = geno_codes_np(spec, np.arange(n_markers))
    G = np.where(codes == 3, np.nan, codes.astype(np.float64))
    Y64 = Y.astype(np.float64)
    t0 = time.perf_counter()
    oracle.scan(G, C, Y64)
    dt = time.perf_counter() - t0
    P = spec.panels[0].n_pheno
    return {
        "value": n_markers * P / dt,
        "unit": "tests/s",
        "cores": blas_threads(),
        "kind": "oracle",
        "sample": f"markers [0, {n_markers}) x all {P} phenotypes at N={spec.n_samples}, K={spec.panels[0].n_cov}; "
                  f"decode, impute, QR, panel prep, explicit residualization, FP64 GEMM, t, p; {dt:.1f} s",
        "seconds": dt,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg3", choices=["cfg2", "cfg3", "cfg4"])
    ap.add_argument("--precision", default="split", choices=["split", "fp32"])
    ap.add_argument("--fp32-steps", type=int, default=1, help="timed steps of the FP32 scan beside (0 = skip)")
    ap.add_argument("--markers", type=int, default=0, help="override M (0 = the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-markers", type=int, default=2048)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--out-budget-gb", type=float, default=60.0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the scan shards by phenotype "
              "columns across GPUs without collectives, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2604_21095_amd import tgw
    from synth import cohort_spec, packed_rows_torch, panel_inputs, row_bytes_for

    torch.cuda.set_device(0)
    tgw.init()
    spec = cohort_spec(args.workload)
    if args.markers:
        spec = spec.__class__(**{**spec.__dict__, "n_markers": args.markers})
    N, M = spec.n_samples, spec.n_markers
    ps = spec.panels[0]
    P, K = ps.n_pheno, ps.n_cov

    # ---------------------------------------------------------------- inputs
    t0 = time.perf_counter()
    geno = torch.empty((M, row_bytes_for(N)), dtype=torch.uint8, device="cuda")
    packed_rows_torch(spec, 0, M, "cuda", out=geno, chunk=8192)
    C, Y = panel_inputs(spec)
    Cd = torch.from_numpy(C).cuda()
    Yd = torch.from_numpy(Y).cuda()
    torch.cuda.synchronize()
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s: N={N} M={M} P={P} K={K}")

    ring = int(max(1024, min(M, args.out_budget_gb * 1e9 / (P * 20))))
    outs = tgw.make_outputs([P], ring)
    stream = torch.cuda.current_stream()

    def one_step(precision, plan_ref, profile=False):
        cov = tgw.fit_covariates(Cd)
        panel = tgw.prepare_phenotypes(cov, Yd, precision)
        plan = tgw.Plan([panel], tile=args.tile)
        if profile:
            plan.profile(True)
        for m0 in range(0, M, ring):
            m1 = min(M, m0 + ring)
            plan.scan(geno, outs, m0, m1)
        plan_ref.append(plan)
        return plan

    def timed(precision, steps, warmup, profile):
        plans = []
        for _ in range(warmup):
            one_step(precision, plans).check()
        plans.clear()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            one_step(precision, plans, profile)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        n_tail = plans[-1].check()
        prof = [p.profile_read() for p in plans] if profile else []
        return dt, n_tail, prof, plans[-1]

    # ---------------------------------------------------------------- autotune
    if not args.no_autotune and args.tile < 0:
        cov = tgw.fit_covariates(Cd)
        panel = tgw.prepare_phenotypes(cov, Yd, args.precision)
        plan = tgw.Plan([panel])
        mt = min(M, ring, 131072)
        best = plan.autotune(geno, outs, 0, mt)
        log(f"autotune: tile {plan.info()['tile']} best {best:.2f} ms on {mt} markers")

    dt, n_tail, prof, plan = timed(args.precision, args.steps, args.warmup, True)
    info = plan.info()
    tile_m, tile_p, waves = tgw.tile_shape(info["tile"])
    tests = M * P
    main_ms = sum(p[0] for p in prof)
    launches = sum(p[1] for p in prof)
    avg_launch_s = main_ms / 1e3 / max(1, launches)
    markers_per_launch = M / (launches / len(prof)) if launches else M
    flops_per_launch = 2.0 * N * markers_per_launch * P
    achieved = flops_per_launch / avg_launch_s / 1e12
    peak = PEAK_BF16_TFLOPS if args.precision == "split" else PEAK_FP32_TFLOPS
    log(f"{args.precision}: {dt * 1e3:.1f} ms/step, {tests / dt:.3e} tests/s, main kernel {avg_launch_s * 1e3:.2f} ms "
        f"x {launches // len(prof)} launches, {achieved:.1f} TFLOP/s algorithmic, tail {n_tail}")

    # ---------------------------------------------------------------- FP32 beside
    fp32 = None
    if args.fp32_steps > 0 and args.precision == "split":
        dt32, _, prof32, _ = timed("fp32", args.fp32_steps, 0, True)
        ms32 = sum(p[0] for p in prof32) / max(1, sum(p[1] for p in prof32))
        fp32 = {"value": tests / dt32, "ms_per_step": dt32 * 1e3, "main_kernel_ms": ms32,
                "main_kernel_tflops": flops_per_launch / (ms32 / 1e3) / 1e12,
                "roofline_frac": flops_per_launch / (ms32 / 1e3) / 1e12 / PEAK_FP32_TFLOPS}
        log(f"fp32: {dt32 * 1e3:.1f} ms/step, {tests / dt32:.3e} tests/s")

    # ---------------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(spec, min(args.cpu_markers, M))
        log(f"cpu oracle: {cpu['value']:.3e} tests/s on {cpu['cores']} threads ({cpu['seconds']:.1f} s)")

    traffic = load_traffic(args.workload, args.precision)
    line = {
        "metric": METRIC,
        "value": tests / dt,
        "unit": "tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if args.precision == "split" else "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: N={N} M={M} P={P} K={K}, 1% missing, 2-bit packed, "
                        f"{'split BF16 hi+lo' if args.precision == 'split' else 'FP32'} contraction",
            "n_samples": N, "n_markers": M, "n_pheno": P, "n_cov": K,
            "precision": args.precision,
            "tile": {"index": info["tile"], "markers": tile_m, "cols": tile_p, "waves": waves},
            "block_markers": info["block_markers"],
            "output_ring_markers": ring,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "kernel": "gemm_kernel (contraction + fused epilogue)",
            "algorithmic_flops_per_launch": flops_per_launch,
            "avg_launch_ms": avg_launch_s * 1e3,
        },
        "cpu_baseline": None if cpu is None else {k: v for k, v in cpu.items() if k != "seconds"},
        "fp32_scan": fp32,
        "tail_tests": n_tail,
        "context": PAPER_CONTEXT,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
