#!/usr/bin/env python
"""Benchmark: superblock Hv/s and Lanczos time to |dE| <= 1e-10 on one MI355X.

One step = one complete ground-state solve of the superblock (every row of the
hot path: the grouped-GEMM Hv H_l V + V H_r^T, the central term, the FP64
Lanczos recurrence with full reorthogonalisation, the tridiagonal eigensolve
and the FP64 residual-corrected restarts) from the seeded start vector to the
solver's convergence, with FP32-MFMA inner products (mixed precision).
value = Hv applications of the K timed solves (FP32 + FP64) / wall time.

Also reported: the same solve on the pure FP64 path, time to energy (the
solver's own stop, and the first restart within 1e-10 of the oracle energy),
Hv-only rates per precision, the roofline of the dominant kernel (grouped
GEMM, timed with HIP events on its stream), and the CPU oracle's Hv rate.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_0707_0159_amd", "csrc", "kernels_hv.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record(workload: str, prec: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "hv_gemm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        recs = json.load(f)
    for r in recs:
        if r.get("workload") == workload and r.get("prec") == prec and r.get("src_hash") == kernel_source_hash():
            return float(r["bytes_per_launch"])
    return None


def cpu_baseline(wl, seconds: float):
    """The oracle's Hv (the paper's matrix form, float64, numpy/scipy) on the host."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import workloads as W
    from oracle.blockio import block_from_arrays
    from oracle.superblock import Superblock

    raw = W.load_blocks(wl.name)
    sb = Superblock(block_from_arrays(raw["L"]), block_from_arrays(raw["R"]), wl.target)
    v = W.random_vector(sb.N, 1000)
    sb.hv_factored(v)                      # builds the dense sectors and the V_c gather plan
    n = 0
    t0 = time.perf_counter()
    while True:
        sb.hv_factored(v)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds or n >= 200:
            break
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": n / dt, "unit": "Hv/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} oracle Hv (mode F: H_l V + V H_r^T + H_c V_c, float64) on {wl.name}, "
                      f"N={sb.N}, {dt:.1f} s, BLAS threads {threads}, host cpus {len(os.sched_getaffinity(0))}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--k-in", type=int, default=24)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", choices=["hv", "copy"], default=None,
                    help="profiling runs for rocprofv3: 'hv' = only Hv launches of --prec, "
                         "'copy' = a plain device copy of known size (counter calibration)")
    ap.add_argument("--prec", choices=["fp64", "fp32"], default="fp32")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the superblock would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_0707_0159_amd import d2d

    if args.profile == "copy":
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "copy", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes}))
        return

    wl = W.CONFIGS[args.config]
    ref_path = os.path.join(ROOT, "tests", "golden", "reference_energies.json")
    E0 = None
    if os.path.exists(ref_path):
        with open(ref_path) as f:
            E0 = json.load(f).get(wl.name, {}).get("E0")

    ctx = d2d.d2d_ctx_create(0)
    raw = W.load_blocks(wl.name)
    model = d2d.make_model(wl.kind, wl.legs, wl.t, wl.U, wl.J)
    b1 = d2d.d2d_block_import(ctx, model, raw["L"])
    b4 = d2d.d2d_block_import(ctx, model, raw["R"])
    sb = d2d.d2d_sb_create(ctx, b1, b4, model, wl.target, (1 << d2d.D2D_FP64) | (1 << d2d.D2D_FP32))
    info = d2d.d2d_sb_info(sb)
    N = info["n"]
    s = ctx.stream
    shapes = d2d.d2d_tile_shapes()
    tuned = {}
    for name, prec in (("fp64", d2d.D2D_FP64), ("fp32", d2d.D2D_FP32)):
        t, ms_t = d2d.d2d_sb_autotune(sb, prec, reps=10)
        tuned[name] = {"tile": t, "BMxBNxBK": "x".join(str(x) for x in shapes[t][1:]), "ms": ms_t}
    with torch.cuda.stream(s):
        v0 = torch.as_tensor(W.random_vector(N, wl.seed), device="cuda")
        psi = torch.zeros_like(v0)
    s.synchronize()

    if args.profile == "hv":
        prec = d2d.D2D_FP32 if args.prec == "fp32" else d2d.D2D_FP64
        with torch.cuda.stream(s):
            x = torch.as_tensor(W.random_vector(N, 1000), device="cuda")
            x = x.float() if prec == d2d.D2D_FP32 else x
            w = torch.empty_like(x)
        for _ in range(args.steps):
            d2d.d2d_hv(sb, prec, x, w)
        s.synchronize()
        print(json.dumps({"profile": "hv", "prec": args.prec, "workload": wl.name, "launches": args.steps,
                          "flops_exec": info["flops_exec"], "bytes_min": info["bytes_min_" + args.prec]}))
        return

    def solve(prec):
        opts = d2d.lanczos_opts(prec=prec, k_in=args.k_in, max_restarts=500, tol_res=args.tol, use_graph=1)
        st, e, stats = d2d.d2d_lanczos(sb, opts, v0, psi)
        if st != 0:
            raise RuntimeError(f"Lanczos did not converge: {stats['residual']}")
        return e, stats

    def first_within(stats, tol=1e-10):
        if E0 is None:
            return None
        for t, th in zip(stats["log_t"], stats["log_theta"]):
            if abs(th - E0) <= tol * abs(E0):
                return t
        return None

    # ---------------------------------------------------------------- timed: mixed precision
    for _ in range(args.warmup):
        solve(d2d.D2D_FP32)
    torch.cuda.synchronize()
    hv = 0
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        e, stats = solve(d2d.D2D_FP32)
        hv += sum(stats["hv_count"])
        last = (e, stats)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e_mixed, st_mixed = last

    # ---------------------------------------------------------------- FP64 path, same algorithm
    solve(d2d.D2D_FP64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    reps64 = max(1, min(args.steps, 5))
    for _ in range(reps64):
        e64, st64 = solve(d2d.D2D_FP64)
    torch.cuda.synchronize()
    wall64 = (time.perf_counter() - t1) / reps64

    # ---------------------------------------------------------------- Hv-only and kernel timing
    with torch.cuda.stream(s):
        x64 = torch.as_tensor(W.random_vector(N, 1000), device="cuda")
        x32 = x64.float()
        w64 = torch.empty_like(x64)
        w32 = torch.empty_like(x32)
    s.synchronize()
    ms = {}
    for name, prec, x, w in (("fp64", d2d.D2D_FP64, x64, w64), ("fp32", d2d.D2D_FP32, x32, w32)):
        d2d.d2d_hv_profile(sb, prec, x, w, reps=5)
        g, c = d2d.d2d_hv_profile(sb, prec, x, w, reps=50)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        for _ in range(50):
            d2d.d2d_hv(sb, prec, x, w)
        ev1.record(s)
        s.synchronize()
        ms[name] = {"gemm_ms": g, "central_ms": c, "hv_ms": ev0.elapsed_time(ev1) / 50}

    F = info["flops_exec"]
    g32 = ms["fp32"]["gemm_ms"] * 1e-3
    achieved = F / g32
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp32"], "traffic": traffic_record(wl.name, "fp32"),
                "kernel": f"k_hv_gemm<float,{tuned['fp32']['BMxBNxBK']}> (grouped GEMM H_l V + V H_r^T, FP32 MFMA 32x32x2)",
                "flops_per_launch": F, "launch_ms": ms["fp32"]["gemm_ms"]}

    line = {
        "metric": "Hv/sec + Lanczos time to |dE|<=1e-10: mixed-precision vs FP64, 1 GPU",
        "value": hv / wall,
        "unit": "Hv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": wl.name, "description": wl.description, "N_sb": N,
                   "sector_pairs": info["npairs"], "m": info["m"], "column_dim": info["ncol"],
                   "central_terms": info["nterms"], "k_in": args.k_in, "tol_res": args.tol,
                   "tiles": tuned,
                   "parallelism": "none (1 GPU)"},
        "time_to_energy": {
            "mixed_s": st_mixed["seconds"], "fp64_s": wall64,
            "speedup_vs_fp64": wall64 / st_mixed["seconds"],
            "mixed_first_within_1e-10_s": first_within(st_mixed),
            "fp64_first_within_1e-10_s": first_within(st64),
            "E_mixed": e_mixed, "E_fp64": e64, "E_oracle": E0,
            "dE_rel_mixed": None if E0 is None else abs(e_mixed - E0) / abs(E0),
            "dE_rel_fp64": None if E0 is None else abs(e64 - E0) / abs(E0),
            "restarts_mixed": st_mixed["restarts"], "hv_count_mixed": st_mixed["hv_count"],
            "restarts_fp64": st64["restarts"], "hv_count_fp64": st64["hv_count"],
        },
        "hv_only": {k: {"hv_per_s": 1e3 / v["hv_ms"], **v} for k, v in ms.items()},
        "flops_exec_per_hv": F, "flops_nnz_per_hv": info["flops_nnz"],
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    d2d.d2d_sb_destroy(sb)
    d2d.d2d_block_destroy(b1)
    d2d.d2d_block_destroy(b4)
    d2d.d2d_ctx_destroy(ctx)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
