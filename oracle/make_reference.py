"""Reference ground energies of the frozen workloads (test infrastructure).

For each workload: load the frozen blocks, build the superblock of Eq. (1)
with the oracle, and find its lowest eigenvalue in the target sector to about
1e-13 relative:

* small targets (N <= 2e6): the oracle Lanczos with full reorthogonalisation,
  checked against ARPACK (``eigsh``, tol=0) on the same operator;
* large targets: ARPACK on the mode-F product, tol=0.

Writes ``tests/golden/reference_energies.json`` (merging with what is there).
Calls only ``oracle/`` and ``workloads``.

    python -m oracle.make_reference --workload heisenberg_2x6_m16 hubbard_2x16_U8_m256
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

import workloads as W

from .blockio import block_from_arrays
from .lanczos import ground_state, ground_state_arpack, kato_temple_lower, lowest_two_arpack
from .lattice import lattice_hamiltonian
from .superblock import Superblock

GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                      "reference_energies.json")


def superblock_of(wl: W.Workload) -> Superblock:
    raw = W.load_blocks(wl.name)
    return Superblock(block_from_arrays(raw["L"]), block_from_arrays(raw["R"]), wl.target)


def reference(wl: W.Workload, ncv=32):
    t0 = time.time()
    sb = superblock_of(wl)
    rec = {"name": wl.name, "target": list(wl.target), "N": int(sb.N), "npairs": len(sb.sectors),
           "block_hash": W.block_file_hash(wl.name)}
    v0 = W.random_vector(sb.N, wl.seed)
    if sb.N <= 2_000_000:
        e1, x1, i1 = ground_state(sb.hv_factored, sb.N, v0=v0, tol=1e-15, max_iter=1500)
        e2, x2, i2 = ground_state_arpack(sb.hv_factored, sb.N, v0=v0, ncv=ncv)
        rec.update(E0=float(e2), E0_lanczos=float(e1), lanczos_iters=i1["iterations"],
                   residual=float(i2["residual"]), agree=float(abs(e1 - e2)))
    else:
        # ARPACK for the two lowest pairs: the second gives the gap of the
        # Kato-Temple bracket  theta - rho^2 / (b - theta) <= E0 <= theta, with
        # b = theta_1 - rho_1 <= lambda_1 (an eigenvalue lies within rho_1 of
        # theta_1, and theta_1 is the second Ritz value)
        e0, e1, x0, r0, r1 = lowest_two_arpack(sb.hv_factored, sb.N, v0=v0, ncv=ncv)
        rec.update(E0=e0, residual=r0, E1=e1, residual1=r1,
                   E0_kato_temple_lower=kato_temple_lower(e0, r0, e1 - r1))
    if wl.nsites <= 16 and wl.kind == "heisenberg":
        H, _ = lattice_hamiltonian(sb.model, wl.length, wl.target)
        rec["E0_lattice_ed"] = float(np.linalg.eigvalsh(H.toarray())[0]) if H.shape[0] <= 6000 else None
    rec["seconds"] = time.time() - t0
    return rec


def second_figure(wl: W.Workload, rec: dict, ncv=32):
    """A second, independent figure for a reference that rests on one ARPACK
    run: the two lowest eigenpairs from a new ARPACK run with their residual
    norms, and the Kato-Temple bracket  theta - rho^2 / (b - theta) <= E0 <= theta
    with b = theta_1 - rho_1."""
    sb = superblock_of(wl)
    v0 = W.random_vector(sb.N, wl.seed + 7)
    e0, e1, x0, r0, r1 = lowest_two_arpack(sb.hv_factored, sb.N, v0=v0, ncv=ncv)
    rec = dict(rec)
    rec.update(E0_second=e0, residual_second=r0, E1=e1, residual1=r1,
               E0_kato_temple_lower=kato_temple_lower(e0, r0, e1 - r1))
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", nargs="+", required=True, choices=sorted(W.WORKLOADS) + ["batch64"])
    ap.add_argument("--length", type=int, default=None, help="batch64 only: lattice length (columns)")
    ap.add_argument("--only", default=None, help="batch64 only: comma-separated problem indices")
    ap.add_argument("--second", action="store_true",
                    help="add the second figure (Kato-Temple bracket) to existing records that lack one")
    args = ap.parse_args()
    data = {}
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            data = json.load(f)
    for name in args.workload:
        wls = W.batch64(args.length) if name == "batch64" else [W.WORKLOADS[name]]
        if name == "batch64" and args.only:
            wls = [wls[int(i)] for i in args.only.split(",")]
        for wl in wls:
            if args.second:
                rec = data.get(wl.name)
                if rec and rec.get("block_hash") == W.block_file_hash(wl.name) and "E0_kato_temple_lower" not in rec:
                    rec = second_figure(wl, rec)
                    print(rec, flush=True)
                    store(wl.name, rec)
                continue
            if wl.name in data and data[wl.name].get("block_hash") == W.block_file_hash(wl.name):
                continue
            pool = W.batch64(args.length) if name == "batch64" else wls
            twin = next((o for o in pool if o.name != wl.name and o.name in data and o.target == wl.target
                         and data[o.name].get("block_hash") == W.block_file_hash(wl.name)), None)
            if twin is not None:
                # the same blocks and target: the same superblock, the same reference
                rec = dict(data[twin.name], name=wl.name, copied_from=twin.name)
                print(f"{wl.name}: reference of {twin.name} (identical superblock)", flush=True)
                store(wl.name, rec)
                continue
            rec = reference(wl)
            print(rec, flush=True)
            store(wl.name, rec)


def store(name: str, rec: dict):
    """Merge one record into the golden file under an exclusive lock (several
    runs of this script may write it at once)."""
    import fcntl
    with open(GOLDEN + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        data = {}
        if os.path.exists(GOLDEN):
            with open(GOLDEN) as f:
                data = json.load(f)
        data[name] = rec
        tmp = GOLDEN + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, GOLDEN)
        fcntl.flock(lk, fcntl.LOCK_UN)


if __name__ == "__main__":
    main()
