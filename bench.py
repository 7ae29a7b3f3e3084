#!/usr/bin/env python
"""Benchmark: superblock Hv/s and Lanczos time to |dE| <= 1e-10 on one MI355X.

One step = one complete ground-state solve of the superblock (every row of the
hot path: the grouped-GEMM Hv H_l V + V H_r^T, the central term, the FP64
Lanczos recurrence with reorthogonalisation, the tridiagonal eigensolve and
the FP64 residual-corrected restarts) from the seeded start vector to the
solver's convergence.  The headline path runs its inner Hv in FP32 on the
matrix cores (mixed precision); value = Hv applications of the K timed solves
(FP32 + FP64) / wall time.

Also reported, on the same algorithm: the BF16-input path (escalating to FP32
if it stalls) and the pure FP64 path; time to energy of each (the solver's own
stop, and the first restart within 1e-10 of the oracle energy); Hv-only rates
per precision; the roofline of the dominant kernel (the grouped GEMM, timed
with HIP events on the stream it runs on) and of the BF16 GEMM; and the CPU
oracle's Hv rate on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME | --config I]

The default workload is the largest single superblock, the 4-leg Heisenberg
ladder 4x16 (m = 1000, N = 4.2e7).  --config indexes
the benchmark set in its fixed order (1 heisenberg_2x6_m16, 2
hubbard_2x16_U8_m256, 3 hubbard_3x12_U4_N33_m400, 4 heisenberg_4x16_m1000,
5 batch64); batch64 runs the batch of 64 uneven superblocks instead (one
grouped launch per Lanczos step over every problem; value = problem Hv
applications per second, summed over the batch).
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

# BF16x3 forms three bf16 products per product: its peak in useful flops is a third of BF16's
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "bf16x3": 2.5e15 / 3, "hbm": 8.0e12}


BASIS_NAMES = {0: "the products' input precision (FP32; BF16 for BF16 products; start vector in FP64)",
               1: "FP64 at every precision", 2: "FP32 below FP64 (start vector in FP64)"}


def step_reads(args) -> int:
    """Reads of the product and the window per Lanczos step in the time model."""
    return 1 if args.one_kernel_step else 2


def basis_name(args):
    return BASIS_NAMES[args.basis]


def basis_bytes(p: int, basis: int) -> int:
    """Bytes per inner basis element for precision index p (0 FP64, 1 FP32, 2 BF16, 3 BF16x3)."""
    if p == 0 or basis == 1:
        return 8
    return 2 if (p == 2 and basis == 0) else 4


PREC_NAMES = ("fp64", "fp32", "bf16", "bf16x3")


def solve_time_parts(stats: dict, n: int, k_in: int, window: int, basis: int, hv_flops: dict,
                     hv_bytes: dict, step_reads: int = 2) -> dict:
    """Lower-bound pieces of one problem's solve (seconds): every Hv at
    max(flops / MFMA peak, minimum bytes / HBM peak) of its precision
    ("hv_s"), the same flops and bytes summed separately ("hv_flop_s",
    "hv_byte_s"), and the Lanczos vector kernels' algorithmic bytes at HBM peak
    ("vec_s").  Per inner step with window w and basis bytes bq (basis_bytes),
    product bytes bw (8 at FP64, else 4): the two step kernels read the
    product twice and the window twice and write the next basis vector, and
    an input copy where the basis is not in the input precision (ci bytes):
    N (2 bw + 2 w bq + bq + ci).  With step_reads = 1 (the one-kernel step,
    which holds its elements in registers across its grid barrier) the product
    and the window count once; that is also a lower bound for a run where some
    steps fall back to the two kernels.  Per restart (FP64 residual, Ritz vector,
    normalisation, first basis vectors): N (88 + (k_in + 1) bq)."""
    hv = stats["hv_count"]
    restarts = stats["restarts"]
    nq = window if window >= 2 else (k_in + 1) / 2.0
    t_hv = t_flop = t_byte = t_step = 0.0
    for p, name in enumerate(PREC_NAMES):
        cnt = hv[p]
        if cnt == 0:
            continue
        tf, tb = hv_flops[name] / PEAK[name], hv_bytes[name] / PEAK["hbm"]
        t_hv += cnt * max(tf, tb)
        t_flop += cnt * tf
        t_byte += cnt * tb
        steps = cnt - (restarts + 1) if p == 0 else cnt     # FP64 counts include the residual products
        bq = basis_bytes(p, basis)
        bw = 8 if p == 0 else 4
        bi = {0: 8, 1: 4, 2: 2, 3: 4}[p]
        ci = 0 if bq == bi else bi
        t_step += max(steps, 0) * n * (step_reads * (bw + nq * bq) + bq + ci) / PEAK["hbm"]
    main = max(range(4), key=lambda q: hv[q] if q else hv[0] - (restarts + 1))
    bq_main = basis_bytes(main, basis)
    t_restart = (restarts + 1) * n * (88 + (k_in + 1) * bq_main) / PEAK["hbm"]
    return {"hv_s": t_hv, "hv_flop_s": t_flop, "hv_byte_s": t_byte, "vec_s": t_step + t_restart}


def solve_time_bound(stats: dict, n: int, k_in: int, window: int, basis: int, hv_flops: dict,
                     hv_bytes: dict, step_reads: int = 2) -> dict:
    """Time-to-energy roofline of one solve: its Hv products, each at the
    bound of its precision, plus the Lanczos vector traffic."""
    t = solve_time_parts(stats, n, k_in, window, basis, hv_flops, hv_bytes, step_reads)
    return {"t_min_ms": (t["hv_s"] + t["vec_s"]) * 1e3, "hv_ms": t["hv_s"] * 1e3,
            "lanczos_vectors_ms": t["vec_s"] * 1e3}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_0707_0159_amd", "csrc", "kernels_hv.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


TILE_KEYS = ("BMxBNxBK", "prefetch_depth", "split_k_loops", "xcd_order")


def tile_desc(t: int, shapes) -> dict:
    """Launch configuration of a d2d_sb_set_tile value: the tile shape (with the
    asymmetric split, the H_l V shape and its transposed partner for V H_r^T,
    the next entry of the table), the K-loop split and the flags."""
    from paper_0707_0159_amd import d2d
    sh = t & 0xFFFF
    if t & d2d.D2D_TILE_ASYM:
        split = "asymmetric"
        dims = "x".join(str(x) for x in shapes[sh][1:4]) + " + " + "x".join(str(x) for x in shapes[sh + 1][1:4])
    else:
        split = "halves" if t & d2d.D2D_TILE_SPLIT4 else bool(t & d2d.D2D_TILE_SPLIT)
        dims = "x".join(str(x) for x in shapes[sh][1:4])
    return {"tile": sh, "split_k_loops": split, "central_in_gemm_launch": bool(t & d2d.D2D_TILE_FUSED),
            "xcd_order": bool(t & d2d.D2D_TILE_XCD), "persistent": bool(t & d2d.D2D_TILE_PERSIST),
            "BMxBNxBK": dims, "prefetch_depth": shapes[sh][4]}


def split_words(split) -> str:
    return {True: ", split K-loops", "halves": ", split K-loops (halved)",
            "asymmetric": ", asymmetric split (H_l V and V H_r^T in transposed tiles)"}.get(split, "")


def traffic_record(workload: str, prec: str, tile: dict):
    """HBM bytes per launch of the grouped GEMM from the committed rocprofv3
    counter summary, if it was taken on the current kernel source and in the
    same launch configuration; else None."""
    path = os.path.join(ROOT, "profiles", "hv_gemm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        recs = json.load(f)
    for r in recs:
        if (r.get("workload") == workload and r.get("prec") == prec and r.get("src_hash") == kernel_source_hash()
                and all(r.get("tile", {}).get(k) == tile.get(k) for k in TILE_KEYS)):
            return float(r["bytes_per_launch"])
    return None


TUNE_CACHE = os.path.join(ROOT, "paper_0707_0159_amd", "tune_cache_mi355x.txt")


def use_tune_cache():
    """Launch configurations come from the committed autotuner results for these
    workloads on MI355X (a private copy, since the library appends to the file
    it is given), unless D2D_TUNE_CACHE is set; a workload the file does not
    hold is autotuned."""
    if os.environ.get("D2D_TUNE_CACHE") or not os.path.exists(TUNE_CACHE):
        return
    import atexit
    import shutil
    import tempfile
    fd, path = tempfile.mkstemp(prefix="d2d_tune_", suffix=".txt")
    os.close(fd)
    shutil.copyfile(TUNE_CACHE, path)
    os.environ["D2D_TUNE_CACHE"] = path
    atexit.register(lambda: os.path.exists(path) and os.remove(path))


def cpu_baseline(wl, seconds: float, iterations: int | None = None, E0=None):
    """The oracle's Hv (the paper's matrix form, float64, numpy/scipy) on the
    host, and the oracle's time to the ground energy: its Lanczos (full
    reorthogonalisation, float64) run to its own stop where the vectors fit
    a bounded run (N <= 2e6), else extrapolated from `iterations` products:
    per iteration k the measured median Hv plus the reorthogonalisation of
    CGS2 against k vectors at the measured time of one length-N dot product
    (4k + 6 dot-equivalents)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import workloads as W
    from oracle.blockio import block_from_arrays
    from oracle.lanczos import ground_state
    from oracle.superblock import Superblock

    raw = W.load_blocks(wl.name)
    sb = Superblock(block_from_arrays(raw["L"]), block_from_arrays(raw["R"]), wl.target)
    v = W.random_vector(sb.N, 1000)
    sb.hv_factored(v)                      # builds the dense sectors and the V_c gather plan
    n = 0
    times = []
    t0 = time.perf_counter()
    while True:
        t1 = time.perf_counter()
        sb.hv_factored(v)
        times.append(time.perf_counter() - t1)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    out = {"value": n / dt, "unit": "Hv/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{n} oracle Hv (mode F: H_l V + V H_r^T + H_c V_c, float64) on {wl.name}, "
                     f"N={sb.N}, {dt:.1f} s, BLAS threads {threads}, host cpus {len(os.sched_getaffinity(0))}"}
    t_hv = float(np.median(times))
    if sb.N <= 2_000_000:
        t1 = time.perf_counter()
        e, _, inf = ground_state(sb.hv_factored, sb.N, v0=W.random_vector(sb.N, wl.seed), tol=1e-14,
                                 max_iter=600)
        out["time_to_energy"] = {"kind": "measured", "s": time.perf_counter() - t1, "iterations": inf["iterations"],
                                 "dE_rel": None if E0 is None else abs(e - E0) / abs(E0),
                                 "what": "oracle Lanczos, full reorthogonalisation, to its own stop (|dtheta| <= "
                                         "1e-14 |theta|)"}
    elif iterations:
        a = W.random_vector(sb.N, 1)
        b = W.random_vector(sb.N, 2)
        t1 = time.perf_counter()
        for _ in range(5):
            float(a @ b)
        t_dot = (time.perf_counter() - t1) / 5
        k = np.arange(1, iterations + 1)
        t = float(iterations * t_hv + np.sum(4 * k + 6) * t_dot)
        out["time_to_energy"] = {"kind": "extrapolated", "s": t, "iterations": int(iterations),
                                 "median_hv_s": t_hv, "dot_s": t_dot,
                                 "what": "iterations = the GPU FP64 solve's product count to its stop (an "
                                         "unrestarted Lanczos needs at most about as many); per iteration k: the "
                                         "oracle's median Hv + (4k + 6) length-N dot products of CGS2 against k "
                                         "vectors"}
    return out


def cpu_baseline_batch(wls, seconds: float):
    """The oracle's Hv over the problems of a batch, in turn, on the host."""
    from threadpoolctl import threadpool_info

    import workloads as W
    from oracle.blockio import block_from_arrays
    from oracle.superblock import Superblock

    n = 0
    t0 = time.perf_counter()
    dt = 0.0
    names = []
    while dt < seconds and n < len(wls):
        wl = wls[n]
        raw = W.load_blocks(wl.name)
        sb = Superblock(block_from_arrays(raw["L"]), block_from_arrays(raw["R"]), wl.target)
        v = W.random_vector(sb.N, 1000)
        t1 = time.perf_counter()
        sb.hv_factored(v)
        dt += time.perf_counter() - t1     # the product only, not the set-up of each problem
        names.append(wl.name)
        n += 1
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": n / dt, "unit": "problem-Hv/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one oracle Hv (mode F, float64) on each of the first {n} problems of the batch, "
                      f"{dt:.1f} s of products, BLAS threads {threads}, host cpus {len(os.sched_getaffinity(0))}"}


def batch_description(wls, infos) -> str:
    """The batch workload in words, with the problems whose blocks hold fewer
    states than their drawn m (blocks of few columns stay exact)."""
    short = [wl.name for wl, i in zip(wls, infos) if i["m"] < wl.m]
    L = wls[0].length
    txt = (f"batch of {len(wls)} uneven superblocks (2/3-leg Heisenberg and Hubbard), {L}-column lattices, "
           f"blocks of {(L - 2) // 2} columns, drawn m 64..512")
    if short:
        txt += f"; {len(short)} problems have blocks below their drawn m (exact blocks of fewer states)"
    else:
        txt += "; every problem's blocks truncated to its drawn m"
    return txt


def bench_batch(args):
    """64 uneven superblocks in one batch: one grouped launch per Lanczos step."""
    import numpy as np
    import torch

    import workloads as W
    from paper_0707_0159_amd import d2d

    wls = W.batch64()
    ref_path = os.path.join(ROOT, "tests", "golden", "reference_energies.json")
    refs = {}
    if os.path.exists(ref_path):
        with open(ref_path) as f:
            g = json.load(f)
        refs = {wl.name: g[wl.name]["E0"] for wl in wls if wl.name in g}
    ctx = d2d.d2d_ctx_create(0)
    s = ctx.stream
    blocks, sbs = [], []
    for wl in wls:
        raw = W.load_blocks(wl.name)
        model = d2d.make_model(wl.kind, wl.legs, wl.t, wl.U, wl.J)
        b1 = d2d.d2d_block_import(ctx, model, raw["L"])
        b4 = d2d.d2d_block_import(ctx, model, raw["R"])
        blocks += [b1, b4]
        sbs.append(d2d.d2d_sb_create(ctx, b1, b4, model, wl.target, 15))
    infos = [d2d.d2d_sb_info(sb) for sb in sbs]
    b = d2d.d2d_batch_create(ctx, sbs)
    # launch configuration of the batch's grouped launches, per precision
    shapes = d2d.d2d_tile_shapes()
    tiles = {}
    for prec, name in ((d2d.D2D_FP64, "fp64"), (d2d.D2D_FP32, "fp32"), (d2d.D2D_BF16, "bf16"),
                       (d2d.D2D_BF16X3, "bf16x3")):
        t, ms_t = d2d.d2d_batch_autotune(b, prec, 2)
        tiles[name] = dict(tile_desc(t, shapes), tuned_ms=ms_t)
    with torch.cuda.stream(s):
        v0 = [torch.as_tensor(W.random_vector(i["n"], wl.seed), device="cuda") for i, wl in zip(infos, wls)]
    s.synchronize()
    # per problem: the method's flops of one Hv (F_nnz, central term included)
    # and the minimum bytes, per precision
    prob_flops = [{n: i["flops_nnz"] for n in PREC_NAMES} for i in infos]
    prob_bytes = [{n: i["bytes_min_" + n] for n in PREC_NAMES} for i in infos]

    def batch_time_bound(per, prec):
        # the batch runs every problem's flops and bytes: time >= the larger of
        # the summed flop and byte times, plus the vector kernels' bytes
        k = args.k_in_bf16 if prec == d2d.D2D_BF16 and args.k_in_bf16 > 0 else args.k_in
        parts = [solve_time_parts(st, i["n"], k, args.window, args.basis, f, by, step_reads(args))
                 for st, i, f, by in zip(per, infos, prob_flops, prob_bytes)]
        t_hv = max(sum(x["hv_flop_s"] for x in parts), sum(x["hv_byte_s"] for x in parts))
        t_vec = sum(x["vec_s"] for x in parts)
        return {"t_min_ms": (t_hv + t_vec) * 1e3, "hv_ms": t_hv * 1e3, "lanczos_vectors_ms": t_vec * 1e3}

    def solve(prec):
        opts = d2d.lanczos_opts(prec=prec, k_in=args.k_in, max_restarts=500, tol_res=args.tol,
                                use_graph=1 if args.graph else 0,
                                reorth_window=args.window, basis=args.basis,
                                k_in_bf16=args.k_in_bf16, fixed_cycles=int(args.fixed_cycles),
                                one_kernel_step=int(args.one_kernel_step))
        st, e, per = d2d.d2d_batch_lanczos(b, opts, v0)
        if st != 0:
            raise RuntimeError("batched Lanczos did not converge")
        return e, per

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            solve(prec)
        torch.cuda.synchronize()
        hv = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            e, per = solve(prec)
            hv += sum(sum(p["hv_count"]) for p in per)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        dE = [abs(x - refs[wl.name]) / abs(refs[wl.name]) for x, wl in zip(e, wls) if wl.name in refs]
        firsts = []
        for p, wl in zip(per, wls):
            E0 = refs.get(wl.name)
            if E0 is None:
                continue
            ft = next((t for t, th in zip(p["log_t"], p["log_theta"]) if abs(th - E0) <= 1e-10 * abs(E0)), None)
            firsts.append(ft)
        bound = batch_time_bound(per, prec)
        bound["frac"] = bound["t_min_ms"] * 1e-3 / (wall / steps)
        return {"hv_per_s": hv / wall, "s_per_solve": wall / steps, "time_roofline": bound,
                "max_dE_rel": max(dE) if dE else None, "problems_with_reference": len(dE),
                "all_within_1e-10_s": (max(firsts) if firsts and None not in firsts else None),
                "restarts_max": max(p["restarts"] for p in per),
                "hv_per_problem_mean": hv / steps / len(per),
                "hv_per_precision_last_solve": [sum(p["hv_count"][q] for p in per) for q in range(4)]}

    head = timed(d2d.D2D_FP32, args.steps, args.warmup)
    reps = max(1, min(args.steps, 3))
    bf16 = timed(d2d.D2D_BF16, reps, 1)
    bf16x3 = timed(d2d.D2D_BF16X3, reps, 1)
    fp64 = timed(d2d.D2D_FP64, reps, 1)

    # one batched Hv (pack + grouped GEMM + central term) per precision, HIP events on the context stream
    hv_ms = {}
    F = sum(i["flops_exec"] for i in infos)
    Fn = sum(i["flops_nnz"] - i["flops_central"] for i in infos)
    Fx = d2d.d2d_batch_gemm_flops(b, d2d.D2D_FP32)
    for prec, name, dt in ((d2d.D2D_FP64, "fp64", torch.float64), (d2d.D2D_FP32, "fp32", torch.float32),
                           (d2d.D2D_BF16, "bf16", torch.bfloat16), (d2d.D2D_BF16X3, "bf16x3", torch.float32)):
        with torch.cuda.stream(s):
            xs = [v.to(dt) for v in v0]
            ws = [torch.empty(v.numel(), dtype=torch.float64 if prec == 0 else torch.float32, device="cuda")
                  for v in v0]
        s.synchronize()
        d2d.d2d_batch_hv(b, prec, xs, ws)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        for _ in range(20):
            d2d.d2d_batch_hv(b, prec, xs, ws)
        ev1.record(s)
        s.synchronize()
        hv_ms[name] = ev0.elapsed_time(ev1) / 20
    line = {
        "metric": "Hv/sec + Lanczos time to |dE|<=1e-10: mixed-precision vs FP64, 1 GPU",
        "value": head["hv_per_s"], "unit": "Hv/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["s_per_solve"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": batch_description(wls, infos),
                   "N_sb_total": sum(i["n"] for i in infos), "N_sb_max": max(i["n"] for i in infos),
                   "k_in": args.k_in, "k_in_bf16": args.k_in_bf16,
                   "fixed_cycles": bool(args.fixed_cycles), "graphs": bool(args.graph),
                   "one_kernel_step": bool(args.one_kernel_step),
                   "reorth_window": args.window,
                   "tol_res": args.tol,
                   "inner_basis": basis_name(args), "parallelism": "none (1 GPU)"},
        "time_to_energy": {"mixed_fp32": head, "mixed_bf16": bf16, "mixed_bf16x3": bf16x3, "fp64": fp64,
                           "speedup_fp32_vs_fp64": fp64["s_per_solve"] / head["s_per_solve"],
                           "speedup_bf16_vs_fp64": fp64["s_per_solve"] / bf16["s_per_solve"],
                           "speedup_bf16x3_vs_fp64": fp64["s_per_solve"] / bf16x3["s_per_solve"]},
        "tiles": tiles,
        "batched_hv_ms": hv_ms,
        "flops_exec_per_batched_hv": F, "gemm_flops_run_fp32": Fx,
        "roofline": {"bound": "mfma", "achieved": Fn / (hv_ms["fp32"] * 1e-3) / 1e12, "peak": PEAK["fp32"] / 1e12,
                     "unit": "TFLOP/s", "frac": Fn / (hv_ms["fp32"] * 1e-3) / PEAK["fp32"], "traffic": None,
                     "work": "F_nnz of every problem's Hv (GEMM part) per batched Hv",
                     "executed_tflops": Fx / (hv_ms["fp32"] * 1e-3) / 1e12,
                     "frac_exec": Fx / (hv_ms["fp32"] * 1e-3) / PEAK["fp32"],
                     "kernel": "batched Hv launch sequence (fp32 grouped GEMM + central term)"},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(wls, args.cpu_seconds)
    d2d.d2d_batch_destroy(b)
    for sb in sbs:
        d2d.d2d_sb_destroy(sb)
    for bl in blocks:
        d2d.d2d_block_destroy(bl)
    d2d.d2d_ctx_destroy(ctx)
    print(json.dumps(line))


SWEEP_CASES = [
    # Fig. 3a: 5-leg x 10 Heisenberg ladder, S_z = 0; Fig. 3b: 3-leg x 10
    # Hubbard ladder, U/t = 10, 28 fermions (14 up, 14 down); smaller lattices
    # of the infinite phase at the same filling
    {"name": "heisenberg_5x10", "kind": "heisenberg", "legs": 5, "L": 10, "t": 1.0, "U": 0.0,
     "m": [32, 128], "target": lambda ns: (ns // 2, 0)},
    {"name": "hubbard_3x10_U10_N28", "kind": "hubbard", "legs": 3, "L": 10, "t": 1.0, "U": 10.0,
     "m": [64, 256], "target": lambda ns: (int(round(14 * ns / 30)), int(round(14 * ns / 30)))},
]


def bench_sweeps(args):
    """Finite-system sweeps on the lattices of Fig. 3: the ground energy at
    the middle position after each sweep, every step's products with the
    transformed start vector and from a random one, and wall times."""
    import numpy as np
    import torch

    from paper_0707_0159_amd import d2d
    from paper_0707_0159_amd.sweep import finite_sweeps

    ctx = d2d.d2d_ctx_create(0)
    out = []
    nsw = max(1, min(args.steps, 4)) if args.steps else 2
    for case in SWEEP_CASES:
        model = d2d.make_model(case["kind"], case["legs"], case["t"], case["U"], 1.0)
        n_col = 2 ** case["legs"] if case["kind"] == "heisenberg" else 4 ** case["legs"]
        for m in case["m"]:
            # turn where the blocks reach m states (exact below when m is a power of the column dimension)
            l_min = 1
            while n_col ** l_min < m:
                l_min += 1
            t0 = time.perf_counter()
            inf, recs = finite_sweeps(ctx, model, case["L"], m, case["target"], l_min, nsw, prec=d2d.D2D_FP32,
                                      compare_random=True,
                                      log=lambda r: print(json.dumps({k: v for k, v in r.items()
                                                                      if not isinstance(v, list)}), flush=True))
            wall = time.perf_counter() - t0
            mid = [r for r in recs if r["position"] == case["L"] // 2 - 1 and r["direction"] != 1]
            per_sweep = [r["energy"] for r in mid]
            steps = recs[1:]
            out.append({
                "lattice": case["name"], "m": m, "l_min": l_min, "sweeps": nsw,
                "N_middle": recs[0]["N"], "energy_infinite": inf[-1]["energy"],
                "energy_middle_per_sweep": per_sweep,
                "energy_lowest": min(r["energy"] for r in recs),
                "products_transformed_start": int(sum(sum(r["hv_count"]) for r in steps)),
                "products_random_start": int(sum(sum(r["hv_count_random"]) for r in steps)),
                "ms_solve_transformed_start": float(np.sum([r["ms_solve"] for r in steps])),
                "ms_solve_random_start": float(np.sum([r["ms_solve_random"] for r in steps])),
                "ms_density_matrix": float(np.sum([r.get("ms_dm", 0.0) for r in steps])),
                "ms_transform": float(np.sum([r.get("ms_transform", 0.0) for r in steps])),
                "steps": len(recs), "wall_s": wall,
                "truncation_max": max(r["trunc"] for r in recs),
            })
            print(json.dumps(out[-1]), flush=True)
    d2d.d2d_ctx_destroy(ctx)
    print(json.dumps({"sweeps": out, "precision": "FP32-mixed Hv, FP64 residual restarts",
                      "data": "synthetic (no inputs: blocks grown from exact one-column blocks)"}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=4, choices=[1, 2, 3, 4, 5],
                    help="workload by its index in the benchmark set (see the module docstring)")
    ap.add_argument("--workload", default=None,
                    help="workload by name (overrides --config): a single superblock's name or batch64")
    ap.add_argument("--k-in", type=int, default=48, help="Krylov dimension per restart")
    ap.add_argument("--k-in-bf16", type=int, default=24, help="Krylov dimension of BF16 cycles (0: --k-in)")
    ap.add_argument("--graph", dest="graph", action="store_true", default=True,
                    help="capture each restart in a hipGraph once and replay it in later solves (the default)")
    ap.add_argument("--no-graph", dest="graph", action="store_false", help="direct launches")
    ap.add_argument("--fixed-cycles", action="store_true",
                    help="every cycle full length (default: the last cycle fitted to the residual bar)")
    ap.add_argument("--one-kernel-step", action="store_true",
                    help="each Lanczos step as one cooperative kernel where the grid fits "
                         "(default: its two kernels)")
    ap.add_argument("--window", type=int, default=3, help="reorthogonalisation window (0 = full)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--basis", type=int, choices=[0, 1, 2], default=0,
                    help="inner basis storage: 0 the products' input precision, 1 FP64, 2 FP32 below FP64")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", choices=["hv", "copy", "density"], default=None,
                    help="profiling runs for rocprofv3: 'hv' = only Hv launches of --prec, "
                         "'copy' = a plain device copy of known size (counter calibration), "
                         "'density' = one FP32-mixed solve, then the density-matrix call twice per side")
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16", "bf16x3"], default="fp32")
    ap.add_argument("--dmrg-step", action="store_true",
                    help="time the routines of one DMRG step on the workload (the paper's split: exact "
                         "diagonalisation, density-matrix formation, diagonalisation, renormalisation)")
    ap.add_argument("--sweeps", action="store_true",
                    help="finite-system sweeps on the two lattices of Fig. 3 (energy per sweep, the products the "
                         "wavefunction transformation saves, time per step)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(sharding the superblock across GPUs is designed, not built)", file=sys.stderr)
        sys.exit(2)
    use_tune_cache()

    import numpy as np
    import torch

    import workloads as W
    from paper_0707_0159_amd import d2d

    if args.sweeps:
        bench_sweeps(args)
        return

    if args.profile == "copy":
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "copy", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes}))
        return

    name = args.workload or W.BENCH_SET[args.config - 1]
    if name == "batch64":
        bench_batch(args)
        return
    if name not in W.WORKLOADS:
        print(f"unknown workload {name}; known: {', '.join(W.BENCH_SET)}", file=sys.stderr)
        sys.exit(2)
    wl = W.WORKLOADS[name]
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
    sb = d2d.d2d_sb_create(ctx, b1, b4, model, wl.target, 15)
    info = d2d.d2d_sb_info(sb)
    N = info["n"]
    s = ctx.stream
    shapes = d2d.d2d_tile_shapes()
    names = {d2d.D2D_FP64: "fp64", d2d.D2D_FP32: "fp32", d2d.D2D_BF16: "bf16", d2d.D2D_BF16X3: "bf16x3"}
    tuned = {}
    for prec, name in names.items():
        t, ms_t = d2d.d2d_sb_autotune(sb, prec, reps=10)
        tuned[name] = dict(tile_desc(t, shapes), ms=ms_t, gemm_flops=d2d.d2d_sb_gemm_flops(sb, prec))
    with torch.cuda.stream(s):
        v0 = torch.as_tensor(W.random_vector(N, wl.seed), device="cuda")
        psi = torch.zeros_like(v0)
    s.synchronize()

    if args.profile == "hv":
        prec = {"fp64": d2d.D2D_FP64, "fp32": d2d.D2D_FP32, "bf16": d2d.D2D_BF16,
                "bf16x3": d2d.D2D_BF16X3}[args.prec]
        with torch.cuda.stream(s):
            x = torch.as_tensor(W.random_vector(N, 1000), device="cuda")
            if prec in (d2d.D2D_FP32, d2d.D2D_BF16X3):
                x = x.float()
            elif prec == d2d.D2D_BF16:
                x = x.to(torch.bfloat16)
            w = torch.empty(N, dtype=torch.float64 if prec == d2d.D2D_FP64 else torch.float32, device="cuda")
        for _ in range(args.steps):
            d2d.d2d_hv(sb, prec, x, w)
        s.synchronize()
        print(json.dumps({"profile": "hv", "prec": args.prec, "workload": wl.name, "launches": args.steps,
                          "tile": tuned[args.prec], "flops_exec": tuned[args.prec]["gemm_flops"],
                          "bytes_min": info["bytes_min_" + args.prec]}))
        return

    if args.profile == "density":
        # the density-matrix call's kernels (formation, the eigensolver's, renormalisation)
        opts = d2d.lanczos_opts(prec=d2d.D2D_FP32, k_in=args.k_in, max_restarts=500, tol_res=args.tol,
                                reorth_window=args.window)
        st, e, _ = d2d.d2d_lanczos(sb, opts, v0, psi)
        if st != 0:
            raise RuntimeError("Lanczos did not converge")
        out = {"profile": "density", "workload": wl.name, "energy": e}
        for side in (0, 1):
            for rep in range(2):
                blk, te, _, ms = d2d.d2d_density_matrix_timed(sb, psi, side, wl.m)
                d2d.d2d_block_destroy(blk)
                out[f"side{side}_rep{rep}_ms"] = [float(x) for x in ms]
                out[f"side{side}_trunc_err"] = te
        torch.cuda.synchronize()
        print(json.dumps(out))
        return

    def solve(prec):
        opts = d2d.lanczos_opts(prec=prec, k_in=args.k_in, max_restarts=500, tol_res=args.tol,
                                use_graph=1 if args.graph else 0,
                                reorth_window=args.window, basis=args.basis,
                                k_in_bf16=args.k_in_bf16, fixed_cycles=int(args.fixed_cycles),
                                one_kernel_step=int(args.one_kernel_step))
        st, e, stats = d2d.d2d_lanczos(sb, opts, v0, psi)
        if st != 0:
            raise RuntimeError(f"Lanczos did not converge: {stats['residual']}")
        return e, stats

    if args.dmrg_step:
        # One DMRG step's routines on this superblock (the paper's performance
        # split): HMED = the ground-state solve (each path, median of steps),
        # then DMF / DMD / renormalisation of both halves for m kept states.
        out = {"workload": wl.name, "N_sb": N, "m_keep": wl.m}
        for prec, nm in ((d2d.D2D_FP64, "fp64"), (d2d.D2D_FP32, "mixed_fp32"), (d2d.D2D_BF16, "mixed_bf16")):
            solve(prec)
            ts = []
            for _ in range(max(1, args.steps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                solve(prec)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            out["hmed_ms_" + nm] = float(np.median(ts)) * 1e3
        solve(d2d.D2D_FP64)                      # psi: the FP64 ground state
        torch.cuda.synchronize()
        for side in (0, 1):
            for rep in range(2):                 # the first call loads the eigensolver's code
                blk, te, _, ms = d2d.d2d_density_matrix_timed(sb, psi, side, wl.m)
                d2d.d2d_block_destroy(blk)
            out[f"side{side}"] = {"dmf_ms": ms[0], "dmd_ms": ms[1], "renorm_ms": ms[2], "trunc_err": te}
        # both halves in one call (their sectors' eigensolves share the streams)
        for rep in range(2):
            bl, br, te2, ms = d2d.d2d_density_matrix_both(sb, psi, wl.m)
            d2d.d2d_block_destroy(bl)
            d2d.d2d_block_destroy(br)
        out["both_halves"] = {"dmf_ms": ms[0], "dmd_ms": ms[1], "renorm_ms": ms[2], "trunc_err": list(te2)}
        print(json.dumps({"dmrg_step": out}))
        d2d.d2d_sb_destroy(sb)
        d2d.d2d_block_destroy(b1)
        d2d.d2d_block_destroy(b4)
        d2d.d2d_ctx_destroy(ctx)
        return

    def first_within(stats, tol=1e-10):
        if E0 is None:
            return None
        for t, th in zip(stats["log_t"], stats["log_theta"]):
            if abs(th - E0) <= tol * abs(E0):
                return t
        return None

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            solve(prec)
        torch.cuda.synchronize()
        hv = 0
        t0 = time.perf_counter()
        last = None
        for _ in range(steps):
            last = solve(prec)
            hv += sum(last[1]["hv_count"])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        e, st = last
        k_path = args.k_in_bf16 if prec == d2d.D2D_BF16 and args.k_in_bf16 > 0 else args.k_in
        bound = solve_time_bound(st, N, k_path, args.window, args.basis,
                                 {k: info["flops_nnz"] for k in tuned},
                                 {k: info["bytes_min_" + k] for k in tuned}, step_reads(args))
        bound["frac"] = bound["t_min_ms"] * 1e-3 / (wall / steps)
        return {"hv_per_s": hv / wall, "s_per_solve": wall / steps, "E": e,
                "dE_rel": None if E0 is None else abs(e - E0) / abs(E0),
                "first_within_1e-10_s": first_within(st), "restarts": st["restarts"],
                "hv_count": st["hv_count"], "precision_log": st["log_prec"], "time_roofline": bound}

    # ---------------------------------------------------------------- timed: headline mixed path (FP32 MFMA)
    head = timed(d2d.D2D_FP32, args.steps, args.warmup)
    # ---------------------------------------------------------------- same algorithm, BF16 inputs / FP64
    reps = max(1, min(args.steps, 5))
    bf16 = timed(d2d.D2D_BF16, reps, 1)
    bf16x3 = timed(d2d.D2D_BF16X3, reps, 1)
    fp64 = timed(d2d.D2D_FP64, reps, 1)

    # ---------------------------------------------------------------- Hv-only and kernel timing
    with torch.cuda.stream(s):
        x64 = torch.as_tensor(W.random_vector(N, 1000), device="cuda")
        xs = {"fp64": x64, "fp32": x64.float(), "bf16": x64.to(torch.bfloat16), "bf16x3": x64.float()}
        ws = {"fp64": torch.empty_like(x64), "fp32": torch.empty(N, dtype=torch.float32, device="cuda"),
              "bf16": torch.empty(N, dtype=torch.float32, device="cuda"),
              "bf16x3": torch.empty(N, dtype=torch.float32, device="cuda")}
    s.synchronize()
    ms = {}
    for prec, name in names.items():
        d2d.d2d_hv_profile(sb, prec, xs[name], ws[name], reps=5)
        g, c = d2d.d2d_hv_profile(sb, prec, xs[name], ws[name], reps=50)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        for _ in range(50):
            d2d.d2d_hv(sb, prec, xs[name], ws[name])
        ev1.record(s)
        s.synchronize()
        ms[name] = {"gemm_ms": g, "central_ms": c, "hv_ms": ev0.elapsed_time(ev1) / 50}

    F = info["flops_exec"]
    F_nnz_gemm = info["flops_nnz"] - info["flops_central"]

    def roofline(name):
        # achieved: the method's work, 2 flops per nonzero of the H_l and H_r
        # sector blocks times the other side's dimension (F_nnz, GEMM part),
        # over the launch's duration; the flops the launch executes (every K
        # step whose operator tile holds a nonzero) are reported beside it
        sec = ms[name]["gemm_ms"] * 1e-3
        fx = tuned[name]["gemm_flops"]
        achieved = F_nnz_gemm / sec
        return {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[name] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK[name], "traffic": traffic_record(wl.name, name, tuned[name]),
                "work": "F_nnz: 2 x nonzeros of the H_l, H_r sector blocks x the other dimension, per launch",
                "flops_nnz_per_launch": F_nnz_gemm,
                "executed_tflops": fx / sec / 1e12, "frac_exec": fx / sec / PEAK[name],
                "executed_over_nnz": fx / F_nnz_gemm,
                "kernel": f"grouped GEMM H_l V + V H_r^T ({name}, tile {tuned[name]['BMxBNxBK']}"
                          f"{split_words(tuned[name]['split_k_loops'])}, zero operator tiles skipped)",
                "flops_per_launch": fx, "dense_sector_flops": F,
                "dense_equivalent_tflops": F / sec / 1e12, "launch_ms": ms[name]["gemm_ms"],
                "hbm_bytes_min_per_launch": info["bytes_min_" + name],
                "hbm_frac_at_min_bytes": info["bytes_min_" + name] / sec / PEAK["hbm"]}

    line = {
        "metric": "Hv/sec + Lanczos time to |dE|<=1e-10: mixed-precision vs FP64, 1 GPU",
        "value": head["hv_per_s"],
        "unit": "Hv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["s_per_solve"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": wl.name, "description": wl.description, "N_sb": N,
                   "sector_pairs": info["npairs"], "m": info["m"], "column_dim": info["ncol"],
                   "central_terms": info["nterms"], "k_in": args.k_in, "k_in_bf16": args.k_in_bf16,
                   "fixed_cycles": bool(args.fixed_cycles), "graphs": bool(args.graph),
                   "one_kernel_step": bool(args.one_kernel_step),
                   "reorth_window": args.window,
                   "tol_res": args.tol, "inner_basis": basis_name(args), "tiles": tuned,
                   "parallelism": "none (1 GPU)"},
        "precision_schedule": "inner Hv FP32 MFMA (FP32 accumulate); FP64 Lanczos scalars, reorthogonalisation "
                              "arithmetic, tridiagonal solve and FP64-Hv residual at every restart; inner basis "
                              f"stored {basis_name(args)}",
        "time_to_energy": {
            "E_oracle": E0,
            "mixed_fp32": head, "mixed_bf16": bf16, "mixed_bf16x3": bf16x3, "fp64": fp64,
            "speedup_fp32_vs_fp64": fp64["s_per_solve"] / head["s_per_solve"],
            "speedup_bf16_vs_fp64": fp64["s_per_solve"] / bf16["s_per_solve"],
            "speedup_bf16x3_vs_fp64": fp64["s_per_solve"] / bf16x3["s_per_solve"],
        },
        "hv_only": {k: {"hv_per_s": 1e3 / v["hv_ms"], **v} for k, v in ms.items()},
        "flops_exec_per_hv": F, "flops_nnz_per_hv": info["flops_nnz"],
        "roofline": roofline("fp32"),
        "roofline_bf16": roofline("bf16"),
        "roofline_bf16x3": roofline("bf16x3"),
        "roofline_fp64": roofline("fp64"),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, iterations=int(fp64["hv_count"][0]), E0=E0)
        if "time_to_energy" in line["cpu_baseline"]:
            line["time_to_energy"]["speedup_fp32_vs_cpu_oracle"] = (
                line["cpu_baseline"]["time_to_energy"]["s"] / head["s_per_solve"])
    d2d.d2d_sb_destroy(sb)
    d2d.d2d_block_destroy(b1)
    d2d.d2d_block_destroy(b4)
    d2d.d2d_ctx_destroy(ctx)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
