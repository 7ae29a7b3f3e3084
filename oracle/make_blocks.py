"""Write the frozen block files of the truncated workloads (test infrastructure).

Runs the oracle's infinite-system growth (float64, CPU) and stores the final
blocks 1 and 4 under ``workloads/blocks/<name>.npz`` together with a JSON log
of every growth step.  Calls nothing outside ``oracle/`` and ``workloads``.

    python -m oracle.make_blocks --workload hubbard_2x16_U8_m256
    python -m oracle.make_blocks --workload batch64 --problems 0-7 [--length 12]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

import workloads as W

from .blockio import save_block_pair
from .dmrg import infinite_system
from .local import Model


def build(wl: W.Workload, tol=1e-10, verbose=True):
    model = Model(wl.kind, wl.legs, t=wl.t, U=wl.U, J=wl.J)
    t0 = time.time()

    def log(info):
        if verbose:
            print(wl.name, {k: (float(f"{v:.12g}") if isinstance(v, float) else v)
                            for k, v in info.items()}, f"{time.time() - t0:.1f}s", flush=True)

    L, R, hist = infinite_system(model, wl.block_cols, wl.m, wl.target_of_sites, seed=0, tol=tol, log=log)
    os.makedirs(W.BLOCK_DIR, exist_ok=True)
    path = W.block_path(wl.name)
    save_block_pair(path, L, R)
    meta = {"name": wl.name, "block_cols": wl.block_cols, "m": wl.m, "dims": [L.dim, R.dim],
            "sectors": [len(L.sectors()), len(R.sectors())], "hash": W.block_file_hash(wl.name),
            "history": [{k: (float(v) if isinstance(v, (float, np.floating)) else v)
                         for k, v in h.items()} for h in hist],
            "growth_tol": tol, "seconds": time.time() - t0}
    with open(path.replace(".npz", ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    return meta


def identical_done(wl: W.Workload, pool) -> W.Workload | None:
    """A problem of the pool with the same model, legs, length and m whose
    block file exists: the growth is deterministic, so its blocks are this
    problem's blocks (the batch draws repeat Heisenberg problems)."""
    for o in pool:
        if (o.name != wl.name and (o.kind, o.legs, o.length, o.m, o.t, o.U, o.J) ==
                (wl.kind, wl.legs, wl.length, wl.m, wl.t, wl.U, wl.J) and os.path.exists(W.block_path(o.name))):
            return o
    return None


def copy_blocks(src: W.Workload, dst: W.Workload):
    import shutil
    shutil.copyfile(W.block_path(src.name), W.block_path(dst.name))
    with open(W.block_path(src.name).replace(".npz", ".json")) as f:
        meta = json.load(f)
    meta.update(name=dst.name, copied_from=src.name)
    with open(W.block_path(dst.name).replace(".npz", ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(f"{dst.name}: blocks of {src.name} (identical problem)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, choices=sorted(W.WORKLOADS) + ["batch64"])
    ap.add_argument("--problems", default=None, help="batch64 only: a-b range")
    ap.add_argument("--length", type=int, default=None, help="batch64 only: lattice length (columns)")
    ap.add_argument("--only", default=None, help="batch64 only: comma-separated problem indices")
    ap.add_argument("--tol", type=float, default=1e-10)
    args = ap.parse_args()
    if args.workload == "batch64":
        probs = W.batch64(args.length)
        if args.problems:
            a, b = (int(x) for x in args.problems.split("-"))
            probs = probs[a:b + 1]
        if args.only:
            probs = [probs[int(i)] for i in args.only.split(",")]
        for wl in probs:
            if os.path.exists(W.block_path(wl.name)):
                continue
            twin = identical_done(wl, W.batch64(args.length))
            if twin is not None:
                copy_blocks(twin, wl)
                continue
            build(wl, tol=args.tol)
    else:
        print(build(W.WORKLOADS[args.workload], tol=args.tol))


if __name__ == "__main__":
    main()
