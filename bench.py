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


# algorithmic ceiling of each precision form at published dense peaks: the
# split forms run two passes per algorithmic FLOP
FORM_CEILING_TFLOPS = {"split8": 1.0 / (1.0 / 2500.0 + 1.0 / 5000.0), "split": 1250.0, "split16": 1250.0,
                       "fp32": 157.3}
WIDE_TILES = (0, 1, 6)  # persistent LDS-ring kernel shapes (the split forms only)


def load_traffic(workload: str, precision: str, tile: int):
    """HBM bytes per main-kernel launch measured with rocprofv3 counters
    (profiles/traffic_gemm_<precision>_<workload>_tile<tile>.txt, "key: value"
    lines), if the kernel source has not changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_gemm_{precision}_{workload}_tile{tile}.txt")
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                d[k.strip()] = v.strip()
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("tile") != str(tile):
        return None
    try:
        return float(d["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain device-to-device copy of 1 GiB (twice), for scaling the
    FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": x.numel() * 4, "copies": 2}))


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"]
        return max(n) if n else 1
    except Exception:
        return os.cpu_count() or 1


def host_info() -> dict:
    """The host the oracle runs on: CPU model, logical CPUs (all and usable), BLAS library."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": i.get("internal_api"), "version": i.get("version"), "threads": i.get("num_threads")}
                for i in threadpool_info() if i.get("user_api") == "blas"]
    except Exception:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "blas": blas}


def cpu_baseline(spec, n_markers: int):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    three equal marker blocks at the start, middle and end of M, all phenotypes."""
    import numpy as np

    import oracle
    from synth import geno_codes_np, pack_codes_np, panel_inputs, row_bytes_for

    C, Y = panel_inputs(spec)
    M = spec.n_markers
    b = max(1, n_markers // 3)
    starts = [0, max(0, M // 2 - b // 2), max(0, M - b)]
    dt = 0.0
    for s in starts:
        packed = pack_codes_np(geno_codes_np(spec, np.arange(s, s + b)), row_bytes_for(spec.n_samples))
        t0 = time.perf_counter()
        oracle.scan_packed(packed, spec.n_samples, C, Y)
        dt += time.perf_counter() - t0
    P = spec.panels[0].n_pheno
    blocks = ", ".join(f"[{s}, {s + b})" for s in starts)
    return {
        "value": 3 * b * P / dt,
        "unit": "tests/s",
        "cores": blas_threads(),
        "kind": "oracle",
        "sample": f"markers {blocks} x all {P} phenotypes at N={spec.n_samples}, K={spec.panels[0].n_cov}; "
                  f"each block: 2-bit decode, impute, QR, panel prep, explicit residualization, FP64 GEMM, t, p; "
                  f"{dt:.1f} s in total; cores = BLAS threads (the rest of the oracle is single-threaded numpy)",
        "host": host_info(),
        "seconds": dt,
    }


def cpu_baseline_1thread(spec, n_markers: int):
    """The same oracle sample on one BLAS thread."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1, user_api="blas"):
        out = cpu_baseline(spec, n_markers)
    out["cores"] = 1
    return out


def generate_genotypes(spec, torch, packed_rows_torch, row_bytes_for):
    """The workload's packed genotypes, generated on the device in eight
    slices (one progress line each)."""
    N, M = spec.n_samples, spec.n_markers
    geno = torch.empty((M, row_bytes_for(N)), dtype=torch.uint8, device="cuda")
    step = max(1, -(-M // 8))
    for a in range(0, M, step):
        b = min(M, a + step)
        packed_rows_torch(spec, a, b, "cuda", out=geno[a:b], chunk=32768)
        torch.cuda.synchronize()
        log(f"genotypes: {b} / {M} markers")
    return geno


def resident(torch, A):
    """A covariate or phenotype matrix as it stays in HBM: (N, cols) with the
    samples of a column contiguous, the layout the library's fit and preparation
    calls read, so the binding passes it through without a transposed copy."""
    return torch.from_numpy(A).cuda().t().contiguous().t()


def panel_scale_run(args, tgw, torch):
    """cfg4 (N=23,000, M=1,000,000, P=20,480, K=10) in the headline precision with
    reduced outputs (per-phenotype best test + hit list): one warm-up step and
    one timed step, main kernel timed with HIP events."""
    from synth import cohort_spec, packed_rows_torch, panel_inputs, row_bytes_for
    spec = cohort_spec("cfg4")
    N, M = spec.n_samples, spec.n_markers
    t0 = time.perf_counter()
    geno = generate_genotypes(spec, torch, packed_rows_torch, row_bytes_for)
    C, Y = panel_inputs(spec, 0)
    Cd, Yd = resident(torch, C), resident(torch, Y)
    del C, Y
    P = Yd.shape[1]
    best = tgw.make_best([P])
    topk = tgw.make_topk([P], args.topk)[0] if args.topk > 0 else None
    outs = [{"best": best[0]} if topk is None else {"best": best[0], "topk": topk}]
    hits, hit_count = tgw.make_hits(1 << 22)
    log(f"panel scale: inputs generated in {time.perf_counter() - t0:.1f} s: N={N} M={M} P={P}")

    def step(profile):
        cov = tgw.fit_covariates(Cd)
        plan = tgw.Plan([tgw.prepare_phenotypes(cov, Yd, args.precision)], tile=args.tile)
        best[0].zero_()
        if topk is not None:
            topk.zero_()
        hit_count.zero_()
        plan.set_hits(hits, hit_count, args.hit_threshold)
        if profile:
            plan.profile(True)
        plan.scan(geno, outs)
        return plan

    if not args.no_autotune and args.tile < 0:
        p0 = step(False)
        p0.check()
        p0.autotune(geno, outs, 0, min(M, 131072))
    step(False).check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = step(True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_tail = plan.check()
    ms, n = plan.profile_read()
    ms /= max(1, n)
    achieved = 2.0 * N * M * P / (ms / 1e3) / 1e12
    peak = PEAK_FP32_TFLOPS if args.precision == "fp32" else PEAK_BF16_TFLOPS
    out = {"workload": f"cfg4: N={N} M={M} P={P} K={spec.panels[0].n_cov}, reduced outputs (best test, "
                       + (f"top {args.topk}, " if topk is not None else "") + f"hits at -log10 p >= {args.hit_threshold})",
           "value": M * P / dt, "unit": "tests/s", "ms_per_step": dt * 1e3, "main_kernel_ms": ms,
           "main_kernel_tflops": achieved, "roofline_frac": achieved / peak, "tile": plan.info()["tile"],
           "hits": int(hit_count.item()), "tail_tests": n_tail}
    log(f"panel scale: {dt * 1e3:.1f} ms/step, {M * P / dt:.3e} tests/s, main kernel {ms:.1f} ms, "
        f"{achieved:.1f} TFLOP/s algorithmic, {out['hits']} hits")
    del geno, Cd, Yd, best, topk, outs, hits, plan
    torch.cuda.empty_cache()
    return out


def batching_run(args, tgw, torch):
    """The batching form (cfg5): 64 panels of log-uniform P in [32, 4096] and K
    in [3, 20] sharing N = 23,000 x M = 200,000 genotypes, headline precision,
    reduced outputs (best test per phenotype + one hit list).  One plan over all
    panels, autotuned, its scan captured in a HIP graph: one warm-up and one
    timed launch.  Beside it, the same panels one plan at a time (one launch
    sequence each, same tile)."""
    from synth import cohort_spec, packed_rows_torch, panel_inputs, row_bytes_for
    spec = cohort_spec("cfg5")
    N, M = spec.n_samples, spec.n_markers
    t0 = time.perf_counter()
    geno = generate_genotypes(spec, torch, packed_rows_torch, row_bytes_for)
    panels, Ps, Ks = [], [], []
    for j in range(len(spec.panels)):
        C, Y = panel_inputs(spec, j)
        cov = tgw.fit_covariates(resident(torch, C))
        panels.append(tgw.prepare_phenotypes(cov, resident(torch, Y), args.precision))
        Ps.append(Y.shape[1])
        Ks.append(C.shape[1])
        del C, Y
    P = sum(Ps)
    log(f"batching: {len(panels)} panels prepared in {time.perf_counter() - t0:.1f} s: N={N} M={M} sum P={P}")
    bests = tgw.make_best(Ps)
    outs = [{"best": b} for b in bests]
    hits, hit_count = tgw.make_hits(1 << 22)
    plan = tgw.Plan(panels)
    plan.set_hits(hits, hit_count, args.hit_threshold)
    if not args.no_autotune:
        plan.autotune(geno, outs, 0, min(M, 131072))
    graph = plan.graph(geno, outs)

    def reset():
        for b in bests:
            b.zero_()
        hit_count.zero_()

    reset()
    graph.launch()
    plan.check()
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graph.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_tail = plan.check()
    n_hits = int(hit_count.item())
    tile = plan.info()["tile"]
    singles = [tgw.Plan([p], tile=tile) for p in panels]
    for sp, o in zip(singles, outs):  # warm-up
        sp.scan(geno, [o])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sp, o in zip(singles, outs):
        sp.scan(geno, [o])
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t0
    out = {"workload": f"cfg5: N={N} M={M}, {len(panels)} panels, sum P={P}, P {min(Ps)}-{max(Ps)}, "
                       f"K {min(Ks)}-{max(Ks)}, reduced outputs, one graph-captured launch sequence",
           "value": M * P / dt, "unit": "tests/s", "ms": dt * 1e3, "tile": tile, "hits": n_hits,
           "tail_tests": n_tail, "one_panel_at_a_time_ms": dt1 * 1e3, "batched_speedup": dt1 / dt}
    log(f"batching: {dt * 1e3:.1f} ms, {M * P / dt:.3e} tests/s; one panel at a time {dt1 * 1e3:.1f} ms "
        f"({dt1 / dt:.2f}x)")
    del graph, plan, singles, panels, geno, bests, outs, hits
    torch.cuda.empty_cache()
    return out


def dosage_run(args, tgw, torch):
    """The workload's cohort as 8-bit dosages (one byte per sample) over
    args.dosage_markers markers, in args.dosage_precision, reduced outputs:
    autotune on the dosage rows, one warm-up and one timed step with the main
    kernel timed by HIP events."""
    from synth import cohort_spec, dosage8_rows_torch, panel_inputs
    spec0 = cohort_spec(args.workload)
    spec = spec0.__class__(**{**spec0.__dict__, "n_markers": args.dosage_markers})
    N, M = spec.n_samples, spec.n_markers
    t0 = time.perf_counter()
    geno = torch.empty((M, (N + 63) // 64 * 64), dtype=torch.uint8, device="cuda")
    step_m = max(1, -(-M // 4))
    for a in range(0, M, step_m):
        b = min(M, a + step_m)
        dosage8_rows_torch(spec, a, b, "cuda", out=geno[a:b], chunk=16384)
        torch.cuda.synchronize()
        log(f"dosages: {b} / {M} markers")
    C, Y = panel_inputs(spec, 0)
    Cd, Yd = resident(torch, C), resident(torch, Y)
    del C, Y
    P = Yd.shape[1]
    best = tgw.make_best([P])
    hits, hit_count = tgw.make_hits(1 << 20)
    log(f"dosages: inputs generated in {time.perf_counter() - t0:.1f} s: N={N} M={M} P={P}")

    def step(profile):
        cov = tgw.fit_covariates(Cd)
        plan = tgw.Plan([tgw.prepare_phenotypes(cov, Yd, args.dosage_precision)])
        best[0].zero_()
        hit_count.zero_()
        plan.set_hits(hits, hit_count, args.hit_threshold)
        if profile:
            plan.profile(True)
        plan.scan(geno, [{"best": best[0]}], code=tgw.CODE_DOSAGE8)
        return plan

    if not args.no_autotune:
        p0 = step(False)
        p0.check()
        p0.autotune(geno, [{"best": best[0]}], 0, min(M, 131072), code=tgw.CODE_DOSAGE8)
    step(False).check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = step(True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.check()
    ms, n = plan.profile_read()
    ms /= max(1, n)
    achieved = 2.0 * N * M * P / (ms / 1e3) / 1e12
    form = {"split16": "FP16 hi + lo", "split8": "FP16 hi + FP8 lo", "fp32": "FP32"}[args.dosage_precision]
    out = {"workload": f"{args.workload} cohort as 8-bit dosages, N={N} M={M} P={P}, {form}, reduced outputs",
           "value": M * P / dt, "unit": "tests/s", "ms_per_step": dt * 1e3, "main_kernel_ms": ms,
           "main_kernel_tflops": achieved, "roofline_frac": achieved / PEAK_BF16_TFLOPS}
    log(f"dosages: {dt * 1e3:.1f} ms/step, {M * P / dt:.3e} tests/s, main kernel {ms:.1f} ms, "
        f"{achieved:.1f} TFLOP/s algorithmic")
    del geno, Cd, Yd, best, hits, plan
    torch.cuda.empty_cache()
    return out


def complete_calls_run(args, tgw, torch, tile, geno, Cd, Yd):
    """Markers without missing calls take the integer centring c = rint(mu),
    whose operand values cost the matrix cores less power: the headline
    precision and tile over args.complete_markers markers of the workload's
    cohort, once as generated (missing calls at the workload's rate: the
    headline rows) and once regenerated without missing calls, reduced
    outputs (best test), main kernel timed with HIP events (one warm-up and
    two timed scans each, alternating)."""
    from synth import cohort_spec, packed_rows_torch, row_bytes_for
    spec0 = cohort_spec(args.workload)
    M = min(args.complete_markers, geno.shape[0])
    spec = spec0.__class__(**{**spec0.__dict__, "n_markers": M, "miss_rate": 0.0})
    whole = torch.empty((M, row_bytes_for(spec.n_samples)), dtype=torch.uint8, device="cuda")
    packed_rows_torch(spec, 0, M, "cuda", out=whole, chunk=32768)
    torch.cuda.synchronize()
    P = Yd.shape[1]
    best = tgw.make_best([P])[0]
    plan = tgw.Plan([tgw.prepare_phenotypes(tgw.fit_covariates(Cd), Yd, args.precision)], tile=tile)
    times = {"missing": [], "complete": []}
    for rep in range(3):
        for name, g in (("missing", geno), ("complete", whole)):
            plan.profile(True)
            plan.scan(g, [{"best": best}], 0, M)
            plan.check()
            ms, n = plan.profile_read()
            plan.profile(False)
            if rep:
                times[name].append(ms / max(1, n))
    a, b = min(times["missing"]), min(times["complete"])
    out = {"workload": f"{args.workload} cohort, M={M}, {args.precision}, tile {tile}, reduced outputs (best test)",
           "main_kernel_ms_with_missing_calls": a, "main_kernel_ms_without_missing_calls": b,
           "speedup": a / b}
    log(f"complete calls: main kernel {a:.2f} ms with 1% missing calls, {b:.2f} ms without ({a / b:.3f}x)")
    del whole, plan, best
    torch.cuda.empty_cache()
    return out


def bed_stream_run(args, tgw, torch, tile):
    """The headline precision over args.bed_markers markers of the workload's
    cohort streamed from a PLINK 1 .bed file (written to a temporary directory,
    so read back from the page cache): one warm-up call (allocates the pinned
    and device slots) and one timed call of tgw_scan_bed, reduced outputs.
    The timed region includes the file reads, host-to-device copies, the
    device-side sample gather and the scan."""
    import shutil
    import tempfile
    from synth import DOSAGE_TO_PLINK, cohort_spec, geno_codes_torch, pack_codes_torch, panel_inputs
    spec0 = cohort_spec(args.workload)
    spec = spec0.__class__(**{**spec0.__dict__, "n_markers": args.bed_markers})
    N, M = spec.n_samples, spec.n_markers
    raw_bytes = (N + 3) // 4
    d = tempfile.mkdtemp(prefix="tgw_bed_", dir=os.environ.get("TMPDIR", "/tmp"))
    try:
        path = os.path.join(d, "cohort.bed")
        lut = torch.from_numpy(DOSAGE_TO_PLINK).cuda()
        t0 = time.perf_counter()
        with open(path, "wb") as f:
            f.write(bytes([0x6C, 0x1B, 0x01]))
            for a in range(0, M, 32768):
                b = min(M, a + 32768)
                codes = lut[geno_codes_torch(spec, a, b, "cuda").long()]
                f.write(pack_codes_torch(codes, raw_bytes).cpu().numpy().tobytes())
                del codes
        log(f"bed stream: wrote {M} x {raw_bytes} B in {time.perf_counter() - t0:.1f} s")
        C, Y = panel_inputs(spec, 0)
        Cd, Yd = resident(torch, C), resident(torch, Y)
        del C, Y
        P = Yd.shape[1]
        best = tgw.make_best([P])
        hits, hit_count = tgw.make_hits(1 << 20)
        bed = tgw.Bed(path, N)

        def step():
            cov = tgw.fit_covariates(Cd)
            plan = tgw.Plan([tgw.prepare_phenotypes(cov, Yd, args.precision)], tile=tile)
            best[0].zero_()
            hit_count.zero_()
            plan.set_hits(hits, hit_count, args.hit_threshold)
            tgw.scan_bed(plan, bed, [{"best": best[0]}], 0, M, block_markers=args.bed_block,
                         n_threads=args.bed_threads)
            plan.check()

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        dt = time.perf_counter() - t0
        bed.close()
        out = {"workload": f"{args.workload} cohort, N={N} M={M} P={P}, PLINK .bed in the page cache, "
                           f"blocks of {args.bed_block} markers, {args.bed_threads} reader threads, reduced outputs",
               "value": M * P / dt, "unit": "tests/s", "ms": dt * 1e3,
               "file_bytes": 3 + M * raw_bytes, "file_gb_per_s": M * raw_bytes / dt / 1e9}
        log(f"bed stream: {dt * 1e3:.1f} ms, {M * P / dt:.3e} tests/s, file {out['file_gb_per_s']:.1f} GB/s")
        return out
    finally:
        shutil.rmtree(d, ignore_errors=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg3", choices=["cfg2", "cfg3", "cfg4", "cfg5"])
    ap.add_argument("--precision", default="split8", choices=["split", "split16", "split8", "fp32"])
    ap.add_argument("--beside", default="split,split16,fp32",
                    help="other precisions timed on the same workload (comma list, '' = none)")
    ap.add_argument("--beside-steps", type=int, default=1)
    ap.add_argument("--markers", type=int, default=0, help="override M (0 = the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-markers", type=int, default=0, help="0: about 15 s of oracle work (16,384 x 2,048 / P)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=int, default=-1)
    ap.add_argument("--out-budget-gb", type=float, default=60.0)
    ap.add_argument("--outputs", default="dense", choices=["dense", "reduced"],
                    help="dense: r, beta, se, t, -log10 p for every test (ring of rows); reduced: per-phenotype "
                         "best test and a hit list at -log10 p >= --hit-threshold, no dense matrices")
    ap.add_argument("--hit-threshold", type=float, default=7.3)
    ap.add_argument("--topk", type=int, default=10,
                    help="with reduced outputs (and in the panel-scale run): per-phenotype top-k lists too (0 = none)")
    ap.add_argument("--copy-calibration", action="store_true", help="run only the 1 GiB copy used to scale counters")
    ap.add_argument("--no-batching", action="store_true", help="skip the cfg5 batching-form leg")
    ap.add_argument("--dosage-markers", type=int, default=262144,
                    help="markers of the 8-bit dosage run beside the headline (0 = skip)")
    ap.add_argument("--dosage-precision", default="split8", choices=["split16", "split8", "fp32"])
    ap.add_argument("--bed-markers", type=int, default=262144,
                    help="markers of the .bed streaming run beside the headline (0 = skip)")
    ap.add_argument("--complete-markers", type=int, default=262144,
                    help="markers of the run with and without missing calls beside the headline (0 = skip)")
    ap.add_argument("--bed-block", type=int, default=32768)
    ap.add_argument("--bed-threads", type=int, default=8)
    ap.add_argument("--arena-gb", type=float, default=32.0,
                    help="device memory of the library's handles: one torch tensor of this many GiB, handed out "
                         "through tgw_arena (0 = hipMalloc and hipFree per handle)")
    ap.add_argument("--no-panel-scale", action="store_true",
                    help="skip the panel-scale run (cfg4: P=20,480, reduced outputs) reported beside the headline")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); across GPUs the scan would shard "
              "by phenotype columns (each GPU a column range of every panel, the genotype stream replicated), "
              "which needs no collectives", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2604_21095_amd import tgw
    from synth import cohort_spec, packed_rows_torch, panel_inputs, row_bytes_for

    torch.cuda.set_device(0)
    tgw.init()
    # the handles (covariate bases, prepared panels, plans) take their memory
    # from one torch allocation: the library's allocator calls are then host
    # bookkeeping instead of hipMalloc / hipFree, which synchronize the device
    arena = tgw.torch_arena(int(args.arena_gb * 2**30)).register() if args.arena_gb > 0 else None
    spec = cohort_spec(args.workload)
    if args.markers:
        spec = spec.__class__(**{**spec.__dict__, "n_markers": args.markers})
    N, M = spec.n_samples, spec.n_markers
    n_panels = len(spec.panels)
    Ps = [p.n_pheno for p in spec.panels]
    Ks = [p.n_cov for p in spec.panels]
    P, K = sum(Ps), Ks[0]

    # ---------------------------------------------------------------- inputs
    t0 = time.perf_counter()
    geno = generate_genotypes(spec, torch, packed_rows_torch, row_bytes_for)
    Cds, Yds = [], []
    for j in range(n_panels):
        C, Y = panel_inputs(spec, j)
        Cds.append(resident(torch, C))
        Yds.append(resident(torch, Y))
        del C, Y
    torch.cuda.synchronize()
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s: N={N} M={M} panels={n_panels} P={P} K={K}")

    reduced = args.outputs == "reduced"
    if reduced:
        ring = M
        bests = tgw.make_best(Ps)
        outs = [{"best": b} for b in bests]
        topks = tgw.make_topk(Ps, args.topk) if args.topk > 0 else []
        for o, tk in zip(outs, topks):
            o["topk"] = tk
        hits, hit_count = tgw.make_hits(1 << 22)
    else:
        ring = int(max(1024, min(M, args.out_budget_gb * 1e9 / (P * 20))))
        outs = tgw.make_outputs(Ps, ring)
    stream = torch.cuda.current_stream()

    def make_plan(precision, tile):
        covs = [tgw.fit_covariates(c) for c in Cds]
        panels = [tgw.prepare_phenotypes(cv, y, precision) for cv, y in zip(covs, Yds)]
        plan = tgw.Plan(panels, tile=tile)
        if reduced:
            for b in bests:
                b.zero_()
            for tk in topks:
                tk.zero_()
            hit_count.zero_()
            plan.set_hits(hits, hit_count, args.hit_threshold)
        return plan

    def one_step(precision, plan_ref, profile=False):
        plan = make_plan(precision, args.tile)
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
        plan = make_plan(args.precision, -1)
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
    peak = PEAK_FP32_TFLOPS if args.precision == "fp32" else PEAK_BF16_TFLOPS
    log(f"{args.precision}: {dt * 1e3:.1f} ms/step, {tests / dt:.3e} tests/s, main kernel {avg_launch_s * 1e3:.2f} ms "
        f"x {launches // len(prof)} launches, {achieved:.1f} TFLOP/s algorithmic, tail {n_tail}")

    # ---------------------------------------------------------------- prepare alone, PCIe-inclusive rate
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    make_plan(args.precision, info["tile"])
    torch.cuda.synchronize()
    prepare_ms = (time.perf_counter() - t0) * 1e3
    host = torch.empty(geno.shape, dtype=torch.uint8, pin_memory=True)
    host.copy_(geno)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    geno.copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    h2d_s = time.perf_counter() - t0
    del host
    log(f"prepare (fit + prepare + plan) {prepare_ms:.1f} ms; packed genotypes host-to-device {h2d_s * 1e3:.1f} ms "
        f"({geno.numel() / h2d_s / 1e9:.1f} GB/s)")
    side = {"prepare_ms": prepare_ms, "h2d_ms": h2d_s * 1e3, "h2d_gb_per_s": geno.numel() / h2d_s / 1e9,
            "tests_per_s_including_h2d": tests / (dt + h2d_s)}

    # ---------------------------------------------------------------- other precisions beside
    beside = {}
    for prec in [x for x in args.beside.split(",") if x and x != args.precision]:
        if not args.no_autotune and args.tile < 0 and prec != "fp32":
            plan = make_plan(prec, -1)
            plan.autotune(geno, outs, 0, min(M, ring, 131072))
        dtb, _, profb, planb = timed(prec, args.beside_steps, 0, True)
        msb = sum(p[0] for p in profb) / max(1, sum(p[1] for p in profb))
        pk = PEAK_FP32_TFLOPS if prec == "fp32" else PEAK_BF16_TFLOPS
        beside[prec] = {"value": tests / dtb, "ms_per_step": dtb * 1e3, "main_kernel_ms": msb,
                        "main_kernel_tflops": flops_per_launch / (msb / 1e3) / 1e12,
                        "roofline_frac": flops_per_launch / (msb / 1e3) / 1e12 / pk,
                        "tile": planb.info()["tile"]}
        log(f"{prec}: {dtb * 1e3:.1f} ms/step, {tests / dtb:.3e} tests/s, main kernel {msb:.2f} ms")

    # ---------------------------------------------------------------- markers without missing calls
    complete = None
    if args.complete_markers > 0 and not args.markers:
        complete = complete_calls_run(args, tgw, torch, info["tile"], geno, Cds[0], Yds[0])

    # ---------------------------------------------------------------- streamed from a .bed file
    bed_stream = None
    if args.bed_markers > 0 and not args.markers:
        bed_stream = bed_stream_run(args, tgw, torch, info["tile"])

    # ---------------------------------------------------------------- 8-bit dosages
    dosage = None
    if args.dosage_markers > 0 and not args.markers:
        dosage = dosage_run(args, tgw, torch)

    # ---------------------------------------------------------------- batching form (cfg5)
    batching = None
    if not args.no_batching and args.workload == "cfg3" and not args.markers:
        batching = batching_run(args, tgw, torch)

    # ---------------------------------------------------------------- panel scale (P = 20,480)
    panel_scale = None
    if not args.no_panel_scale and args.workload == "cfg3" and not args.markers:
        del outs, geno, Cds, Yds
        plan = planb = None
        torch.cuda.empty_cache()
        panel_scale = panel_scale_run(args, tgw, torch)

    # ---------------------------------------------------------------- CPU baseline
    cpu = cpu1 = None
    if not args.no_cpu_baseline:
        n_cpu = min(args.cpu_markers or max(256, 16384 * 2048 // P), M)
        cpu = cpu_baseline(spec, n_cpu)
        log(f"cpu oracle: {cpu['value']:.3e} tests/s on {cpu['cores']} threads ({cpu['seconds']:.1f} s)")
        cpu1 = cpu_baseline_1thread(spec, max(64, n_cpu // 16))
        log(f"cpu oracle, one thread: {cpu1['value']:.3e} tests/s ({cpu1['seconds']:.1f} s)")

    traffic = load_traffic(args.workload, args.precision, info["tile"])
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
        "dtype": {"split": "bf16", "split16": "fp16", "split8": "fp16+fp8", "fp32": "fp32"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: N={N} M={M} "
                        + (f"P={P} K={K}" if n_panels == 1 else f"{n_panels} panels, sum P={P}, K {min(Ks)}-{max(Ks)}")
                        + f", 1% missing, 2-bit packed, "
                        + {"split": "split BF16 hi+lo", "split16": "split FP16 hi+lo",
                           "split8": "FP16 hi + FP8 e4m3 lo", "fp32": "FP32"}[args.precision]
                        + " contraction",
            "n_samples": N, "n_markers": M, "n_pheno": P, "n_cov": K, "n_panels": n_panels,
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
            "kernel": ("gemm_wide_kernel" if info["tile"] in WIDE_TILES and args.precision != "fp32" else "gemm_kernel")
                      + " (contraction + fused epilogue)",
            "peak_basis": "dense 16-bit MFMA; the FP8 lo pass of split8 runs at twice that rate"
                          if args.precision == "split8" else "dense MFMA of the operand type",
            # the form's own ceiling at published peaks: one FP16 pass (2.5 PFLOP/s) plus one FP8
            # pass (5.0 PFLOP/s) per algorithmic FLOP, 1 / (1/2.5 + 1/5) = 1.67 PFLOP/s
            "form_ceiling": FORM_CEILING_TFLOPS.get(args.precision),
            "frac_of_form_ceiling": achieved / FORM_CEILING_TFLOPS[args.precision]
                                    if args.precision in FORM_CEILING_TFLOPS else None,
            "algorithmic_flops_per_launch": flops_per_launch,
            "avg_launch_ms": avg_launch_s * 1e3,
        },
        "cpu_baseline": None if cpu is None else {k: v for k, v in cpu.items() if k != "seconds"},
        "cpu_baseline_1thread": None if cpu1 is None else {k: v for k, v in cpu1.items() if k != "seconds"},
        "prepare_and_transfer": side,
        "fp32_scan": beside.get("fp32"),
        "split_scan": beside.get("split"),
        "split16_scan": beside.get("split16"),
        "split8_scan": beside.get("split8"),
        "tail_tests": n_tail,
        "panel_scale": panel_scale,
        "bed_stream": bed_stream,
        "dosage8_scan": dosage,
        "complete_calls": complete,
        "batching": batching,
        "device_memory": ("hipMalloc / hipFree per handle" if arena is None else
                          {"kind": "tgw_arena over one torch tensor", "capacity_gib": args.arena_gb,
                           "peak_gib": arena.info().peak / 2**30}),
        "outputs": ("dense r, beta, se, t, -log10 p" if not reduced else
                    f"reduced: per-phenotype best test" + (f" + top {args.topk}" if args.topk > 0 else "")
                    + f" + hit list at -log10 p >= {args.hit_threshold} "
                    f"({int(hit_count.item())} hits in the last step)"),
        "context": PAPER_CONTEXT,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
