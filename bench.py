#!/usr/bin/env python3
"""Throughput of the rank-profile-revealing PLDL^TP^T factorization over F_p on one MI355X.

Metric (Section 6 of the paper): effective GOPS = (r^3/3 + n^2 r - r^2 n) / (1e9 * time),
one step = one whole factorization (pldl_factor: recursive cascade, the products on
the matrix cores of the library's default path, INT8 split for p < 2^23 and FP64
otherwise; --path forces one) of a seeded synthetic matrix already resident in HBM.

Default workload: n = 16384 over F_8388593 with a uniformly random rank profile of
rank 12288 (A = L R L^T, L random unit lower, R a seeded symmetric rook placement).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
PEAK_INT8_TOPS = 5000.0   # MI355X dense INT8 matrix peak
PEAK_HBM_GBS = 8000.0
METRIC = "effective mod-p GOPS (n\u00b2r-normalized), exact"
# HBM traffic of the product kernel per launch, from two rocprofv3 --pmc passes (FETCH_SIZE,
# WRITE_SIZE) scaled by a plain copy of known size; valid only for the kernel sources it
# was measured on (their SHA-256 is recorded beside the figure).
PRODUCT = {
    "f64": dict(kernel="k_gemm", cls="gemm", sources=("paper_1802_10453_amd/csrc/gemm.hip",
                                                      "paper_1802_10453_amd/csrc/common.h")),
    "i8": dict(kernel="k_gemm_i8", cls="gemm_i8", sources=("paper_1802_10453_amd/csrc/gemm_i8.hip",
                                                           "paper_1802_10453_amd/csrc/common.h")),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def eff_ops(n, r):
    return r ** 3 / 3.0 + n * n * r - r * r * n


def cpu_baseline(workload_p):
    """The oracle (plain CPU elimination, OpenMP over the trailing update) on a bounded
    sample of the same input family: n = 4608, rank 3456, random rank profile (about
    10 s of host work on 16 cores)."""
    import oracle.oracle as orc
    from paper_1802_10453_amd import inputs
    n, p = 4608, workload_p
    r = 3456
    A, _ = inputs.rank_profile_matrix_input(n, p, r // 2, r // 4, inputs.SEED_BASE + 100, check=8)
    orc.lib()
    t0 = time.perf_counter()
    res = orc.search(A, p)
    dt = time.perf_counter() - t0
    assert res["rank"] == r
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    return dict(value=eff_ops(n, r) / dt / 1e9, unit="effective GOPS", cores=cores, kind="oracle",
                sample=f"oracle search on n={n} p={p} rank={r} random-RPM input (same generator), {dt:.2f} s")


def source_hash(sources):
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(path, workload, n, p, r):
    """Bytes per product-kernel launch from the committed counter summary, or None when
    it is missing, was taken on another workload, or the kernel sources changed since."""
    pr = PRODUCT[path]
    fn = os.path.join(ROOT, "profiles", f"{pr['kernel']}.n{n}_p{p}_rank{r}.traffic.txt")
    try:
        kv = {}
        with open(fn) as f:
            for line in f:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("workload") != workload or kv.get("sources_sha256") != source_hash(pr["sources"]):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline_batched(mats, params, p, sample=2048):
    """The oracle on the first `sample` matrices of the same batch."""
    import oracle.oracle as orc
    orc.lib()
    t0 = time.perf_counter()
    for A in mats[:sample]:
        orc.search(A, p)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    ops = sum(eff_ops(n, r) for (n, r, f, c, s) in params[:sample])
    return dict(value=sample / dt, unit="factorizations/s", cores=cores, kind="oracle",
                sample=f"oracle search on the first {sample} matrices of the batch ({dt:.2f} s, "
                       f"{ops / dt / 1e9:.3f} effective GOPS)")


def pluq_comparison(ctx, torch, A0, p, ldlt_ms, ldlt_rank, steps=2):
    """The same input factored as an unsymmetric matrix by the rank-profile-revealing
    PLUQ (pldl_plduq, the elimination the symmetric one is compared with in Section 6):
    one warm-up, then `steps` timed calls on fresh FP64 copies."""
    log("[bench] unsymmetric PLUQ of the same input ...")
    copies = [A0.double() for _ in range(steps + 1)]
    out = ctx.plduq(p, copies[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        out = ctx.plduq(p, copies[1 + k])
    torch.cuda.synchronize()
    pms = (time.perf_counter() - t0) * 1e3 / steps
    del copies
    if out["rank"] != ldlt_rank:
        log(f"[bench] PLUQ rank {out['rank']} differs from the factorization's {ldlt_rank}")
        sys.exit(1)
    log(f"[bench] PLUQ {pms:.3f} ms per call, {pms / ldlt_ms:.2f}x the symmetric factorization")
    return dict(pluq_ms_per_step=round(pms, 3), ldlt_ms_per_step=round(ldlt_ms, 3),
                pluq_over_ldlt=round(pms / ldlt_ms, 3), rank=out["rank"], steps=steps,
                entry="pldl_plduq on the same n x n input (FP64 residues)")


def bench_batched(args, torch, inputs, pldl):
    """Batched workload: every step is one replay of a captured graph holding the whole
    persistent batched launch, on its own copy of the input batch."""
    cfg = inputs.C3
    p = cfg["p"]
    workers = min(16, os.cpu_count() or 1) if args.gen_workers < 0 else args.gen_workers
    log(f"[bench] generating {cfg['name']} with {max(workers, 1)} process(es) ...")
    t0 = time.perf_counter()
    mats, params = inputs.batch_input(cfg, workers=workers, progress=lambda k: log(f"[bench]   {k} matrices"))
    log(f"[bench] input ready in {time.perf_counter() - t0:.1f} s")
    ctx = pldl.Context(0)
    nrun = args.warmup + args.steps
    arenas = []
    for k in range(nrun):
        dev = [torch.from_numpy(A.astype(np.int32)).cuda() for A in mats]
        arenas.append(ctx.batched_args(dev))
    # first call outside any capture: allocates the workspace and the inverse table
    scratch = ctx.batched_args([torch.from_numpy(A.astype(np.int32)).cuda() for A in mats[:4]])
    ctx.factor_batched(p, scratch)
    torch.cuda.synchronize()
    graphs = []
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for a in arenas:
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr, stream=s):
                ctx.factor_batched(p, a)
            graphs.append(gr)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for w in range(args.warmup):
        graphs[w].replay()
    torch.cuda.synchronize()
    # correctness of what is timed (warm-up arena): statuses and ranks
    if args.warmup:
        st = arenas[0]["status"].cpu().numpy()
        rk = arenas[0]["rank"].cpu().numpy()
        ok = (st == 0).all() and all(int(rk[t]) == params[t][1] for t in range(len(params)))
        log(f"[bench] statuses and ranks vs generator: {'ok' if ok else 'MISMATCH'}")
        if not ok:
            sys.exit(1)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for k in range(args.steps):
        graphs[args.warmup + k].replay()
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    rk = arenas[-1]["rank"].cpu().numpy()
    if not all(int(rk[t]) == params[t][1] for t in range(len(params))):
        log("[bench] rank mismatch in the timed run")
        sys.exit(1)
    ops = sum(eff_ops(n, r) for (n, r, f, c, s2) in params)
    count = len(mats)
    value = count / (ms / 1e3)
    # the Section 6 count already counts a field multiply and a field add as two
    # operations (n^3/3 at full rank: the flops of symmetric elimination)
    flops = ops
    achieved = flops / (kern_ms / 1e3) / 1e12
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP64_TFLOPS, 4), traffic=None,
                    kernel="k_factor_batched (FP64 vector elimination; peak = 256 CUs x 2.4 GHz x 128 FP64 "
                           "flops/clk)", launches=args.steps, avg_launch_ms=round(kern_ms, 4))
    log(f"[bench] {count} factorizations in {ms:.3f} ms per step ({ops / (ms / 1e3) / 1e9:.1f} effective GOPS)")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline_batched(mats, params, p)
    line = {
        "metric": "batched factorizations/s", "value": round(value, 1), "unit": "factorizations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "count": count, "p": p, "n_range": [cfg["nmin"], cfg["nmax"]],
                   "aggregate_effective_gops": round(ops / (ms / 1e3) / 1e9, 2),
                   "launch": "one persistent kernel per step, replayed from a captured HIP graph",
                   "input": "uint32 residues in HBM"},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--threshold", type=int, default=0)
    ap.add_argument("--gen-workers", type=int, default=-1,
                    help="processes that build the batched input (-1: up to 16, 0: this process)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the base-case threshold with pldl_autotune before the warm-up (untimed)")
    ap.add_argument("--path", default="auto", choices=["auto", "f64", "i8"],
                    help="matrix cores of the products: the library's default (auto: INT8 split for p < 2^23, "
                         "else FP64), FP64 with delayed reduction, or INT8 with residues split into signed bytes")
    ap.add_argument("--no-profile", action="store_true", help="time without per-launch events (no roofline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--winograd", type=int, default=0, metavar="MIN_ORDER",
                    help="dense products with m, n, k >= MIN_ORDER take Winograd levels (pldl_set_winograd; 0: off)")
    ap.add_argument("--no-pluq", action="store_true",
                    help="skip the comparison with the unsymmetric RPM-revealing PLUQ (pldl_plduq) of the same input")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="before the timed steps, run one plain device copy of BYTES bytes (an elementwise "
                         "kernel reading and writing BYTES each): the reference for the HBM counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this library runs one factorization per GPU and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1802_10453_amd import inputs, pldl

    if args.workload == "c3":
        return bench_batched(args, torch, inputs, pldl)
    cfg = {"c1": inputs.C1, "c2": inputs.C2, "c4": inputs.C4}[args.workload]
    n, p = cfg["n"], cfg["p"]
    log(f"[bench] generating {cfg['name']} ...")
    t0 = time.perf_counter()
    A_np, rpm_gen = inputs.config_input(cfg, device="cuda", check=16)
    log(f"[bench] input ready in {time.perf_counter() - t0:.1f} s")
    A0 = torch.from_numpy(A_np.astype(np.int32)).cuda()
    del A_np
    nrun = args.warmup + args.steps + (0 if args.no_profile else 1)
    copies = [A0.clone() for _ in range(nrun)]
    ctx = pldl.Context(0)
    ctx.set_path({"auto": pldl.PLDL_PATH_AUTO, "f64": pldl.PLDL_PATH_F64, "i8": pldl.PLDL_PATH_I8}[args.path])
    ctx.set_winograd(args.winograd)
    threshold_used = args.threshold or 128
    if args.autotune and not args.threshold:
        import tempfile
        tpath = os.path.join(tempfile.mkdtemp(), "tune.txt")
        t0 = time.perf_counter()
        ctx.autotune(p, [n], table_path=tpath)
        with open(tpath) as f:
            row = [l.split() for l in f if not l.startswith("#")][0]
        threshold_used = int(row[2])
        log(f"[bench] autotuned threshold {threshold_used} in {time.perf_counter() - t0:.1f} s "
            f"(uniform {row[3]} ms, rank-profile {row[4]} ms at that threshold)")
    out = None
    for w in range(args.warmup):
        out = ctx.factor(copies[w], p, threshold=args.threshold)
        log(f"[bench] warmup {w} rank {out['rank']}")
    # correctness of what is timed: rank and rank profile against the generator's closed form
    if out is not None and rpm_gen is not None:
        ok = out["rank"] == int((rpm_gen >= 0).sum()) and bool((out["rpm"].cpu().numpy() == rpm_gen).all())
        log(f"[bench] rank/rpm vs generator: {'ok' if ok else 'MISMATCH'}")
        if not ok:
            sys.exit(1)
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.calibrate_copy} bytes read, {args.calibrate_copy} bytes written")
        del src, dst
    torch.cuda.synchronize()
    if not args.no_profile:
        ctx.profile(3)   # events around the GEMM launches only: the roofline kernel
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = ctx.factor(copies[args.warmup + k], p, threshold=args.threshold)
        log(f"[bench] step {k} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = ctx.profile(0) if not args.no_profile else None
    ms = (t1 - t0) * 1e3 / args.steps
    full = None
    if not args.no_profile:
        # per-class breakdown from one more, untimed step with every launch recorded
        ctx.profile(1)
        ctx.factor(copies[-1], p, threshold=args.threshold)
        torch.cuda.synchronize()
        full = ctx.profile(0)
    r = out["rank"]
    sched = out["schedule"]   # of the last timed step: threshold, split rule, path, launches, host waits
    path = "i8" if sched["path_used"] == pldl.PLDL_PATH_I8 else "f64"   # the path the steps took
    value = eff_ops(n, r) / (ms / 1e3) / 1e9
    roofline = None
    if stats is not None:
        pr = PRODUCT[path]
        g = stats[pr["cls"]]
        traffic = measured_traffic(path, cfg["name"], n, p, r)
        if path == "f64":
            achieved = g["flops"] / (g["ms"] / 1e3) / 1e12 if g["ms"] > 0 else 0.0
            roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                            frac=round(achieved / PEAK_FP64_TFLOPS, 4), traffic=traffic,
                            kernel="k_gemm (FP64 MFMA mod-p product)")
        else:
            achieved = g["ops8"] / (g["ms"] / 1e3) / 1e12 if g["ms"] > 0 else 0.0
            roofline = dict(bound="mfma", achieved=round(achieved, 3), peak=PEAK_INT8_TOPS, unit="TOP/s",
                            frac=round(achieved / PEAK_INT8_TOPS, 4), traffic=traffic,
                            kernel="k_gemm_i8 (INT8 MFMA on signed-byte limbs)",
                            modp_tflops=round(g["flops"] / (g["ms"] / 1e3) / 1e12, 3) if g["ms"] > 0 else 0.0)
        roofline["launches"] = g["launches"]
        roofline["avg_launch_ms"] = round(g["ms"] / max(g["launches"], 1), 4)
        # each operand read once, C read and written: the floor `traffic` is compared with
        roofline["alg_bytes_per_launch"] = round(g["bytes"] / max(g["launches"], 1), 1)
    if full is not None:
        tot_ms = sum(v["ms"] for k2, v in full.items() if k2 != "host_sync")
        log("[bench] per-class GPU time of one extra step with every launch event-timed (ms; the events "
            "themselves add queue time):")
        for k2, v in full.items():
            log(f"    {k2:11s} launches {v['launches']:8.0f}  ms {v['ms']:9.3f}"
                + (f"  {v['flops'] / v['ms'] / 1e9:8.2f} mod-p TFLOP/s" if v["flops"] and v["ms"] else "")
                + (f"  {v['ops8'] / v['ms'] / 1e9:8.2f} INT8 TOP/s" if v["ops8"] and v["ms"] else "")
                + (f"  {v['bytes'] / v['ms'] / 1e6:8.1f} GB/s" if v["bytes"] and v["ms"] else ""))
        log(f"    sum of kernel time {tot_ms:.3f} ms; timed steps {ms:.3f} ms/step")
    pluq = None
    if not args.no_pluq:
        pluq = pluq_comparison(ctx, torch, A0, p, ms, r)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(p)
    line = {
        "metric": METRIC,
        "value": round(value, 2), "unit": "GOPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if path == "f64" else "i8", "data": "synthetic",
        "config": {"workload": cfg["name"], "n": n, "p": p, "rank": r, "threshold": sched["threshold_used"],
                   "path": "fp64-mfma" if path == "f64" else "int8-split-mfma",
                   "winograd_min_order": args.winograd, "input": "uint32 residues in HBM", "schedule": sched},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    if pluq is not None:
        line["pluq_comparison"] = pluq
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
