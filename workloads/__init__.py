"""Seeded synthetic workloads shared by the oracle side and the HIP side.

This module holds *no arithmetic of the method*: it names the workloads
(model, lattice, kept states, target quantum numbers), draws seeded random
vectors, and loads the frozen block files as raw arrays.  Both the oracle
(``oracle/``) and the HIP binding read their inputs from here; neither
imports the other.

The paper's workloads are model Hamiltonians fixed by a few parameters; no
dataset is involved.  The frozen block files under ``workloads/blocks`` are
written once by ``oracle/make_blocks.py`` (infinite-system growth in float64
on the CPU) and never by the HIP path.

Block file layout (``numpy.savez``; ``P`` is ``"L_"`` or ``"R_"``):

* ``P+kind``    int: 0 Heisenberg, 1 Hubbard;  ``P+legs``, ``P+ncols``,
  ``P+side`` (0 left block, 1 right block); ``P+t``, ``P+U``, ``P+J``.
* ``P+sec_qn``  int64 ``(nsec, 2)``: ``(n_up, n_dn)`` of each sector, ascending.
* ``P+sec_dim`` int64 ``(nsec,)``.
* ``P+H``       float64: block Hamiltonian, one dense column-major
  ``d x d`` block per sector, in sector order.
* ``P+op_key``  int64 ``(nops, 3)``: edge operator names,
  ``(0, y, sigma)`` = annihilator c_{y,sigma} (Jordan-Wigner string over the
  block's earlier modes folded in), ``(1, y, 0)`` = S^z_y,
  ``(2, y, 0)`` = S^+_y.
* ``P+op_blk``  int64 ``(nblk, 3)``: ``(op index, sector from, sector to)``.
* ``P+op_off``  int64 ``(nblk,)``: offset of each block in ``P+op_data``.
* ``P+op_data`` float64: dense column-major ``d_to x d_from`` blocks.
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass, field
from typing import Callable

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BLOCK_DIR = os.path.join(HERE, "blocks")

KIND_HEISENBERG = 0
KIND_HUBBARD = 1


def _half_filling(legs):
    def f(nsites):
        return (nsites // 2, nsites // 2)
    return f


def _sz_zero(legs):
    def f(nsites):
        return (nsites // 2, 0)
    return f


def _doped_11_12(nsites):
    """N = round-half-even(11/12 * sites), N_up = ceil(N/2)."""
    N = int(round(11 * nsites / 12))          # Python's round is half-even
    nup = (N + 1) // 2
    return (nup, N - nup)


@dataclass
class Workload:
    """One superblock problem: model, lattice, kept states, target sector."""

    name: str
    kind: str                 # "heisenberg" | "hubbard"
    legs: int
    length: int               # columns of the full lattice
    m: int                    # states kept in blocks 1 and 4
    t: float = 1.0
    U: float = 0.0
    J: float = 1.0
    target_of_sites: Callable = field(default=None, repr=False)
    seed: int = 0             # Lanczos start-vector seed
    description: str = ""

    @property
    def block_cols(self) -> int:
        return (self.length - 2) // 2

    @property
    def nsites(self) -> int:
        return self.legs * self.length

    @property
    def target(self):
        return self.target_of_sites(self.nsites)

    @property
    def kind_id(self) -> int:
        return KIND_HUBBARD if self.kind == "hubbard" else KIND_HEISENBERG

    @property
    def column_dim(self) -> int:
        return (4 if self.kind == "hubbard" else 2) ** self.legs


def _batch64_problems(length):
    """64 uneven superblocks: one default_rng(5) stream, drawn problem by problem
    (the draws do not depend on the lattice length)."""
    rng = np.random.default_rng(5)
    out = []
    for i in range(64):
        legs = int(rng.choice([2, 3]))
        kind = str(rng.choice(["hubbard", "heisenberg"]))
        m = int(rng.choice([64, 128, 256, 512]))
        U = float(rng.uniform(2.0, 10.0)) if kind == "hubbard" else 0.0
        tgt = _half_filling(legs) if kind == "hubbard" else _sz_zero(legs)
        out.append(Workload(f"batch{i:02d}_{kind}_{legs}x{length}_m{m}", kind, legs,
                            length, m, t=1.0, U=U, J=1.0, target_of_sites=tgt,
                            seed=100 + i))
    return out


# Lattice length of the batch problems.  At 12 columns the blocks have 5
# columns, more states than any drawn m, so every problem truncates to its m.
# 6 columns (blocks of 2 columns) is the short variant, kept as test input:
# the blocks of its 2-leg and 3-leg Heisenberg problems (16 and 64 states)
# and of its 2-leg Hubbard problems (256 states) are exact, below the larger
# drawn m, so their superblocks are whole lattices that exact
# diagonalisation checks.
BATCH_LENGTH = 12
BATCH_LENGTH_DRAWN = 12

HEISENBERG_2X6_M16 = Workload("heisenberg_2x6_m16", "heisenberg", 2, 6, 16, J=1.0, target_of_sites=_sz_zero(2),
                              description="2-leg Heisenberg ladder 2x6, exact blocks of two rungs (m=16), "
                                          "columns of dim 4, superblock dim 4096")
HUBBARD_2X16_M256 = Workload("hubbard_2x16_U8_m256", "hubbard", 2, 16, 256, t=1.0, U=8.0,
                             target_of_sites=_half_filling(2),
                             description="2-leg Hubbard ladder 2x16, t=1, U=8, half filling, m=256")
HUBBARD_3X12_M400 = Workload("hubbard_3x12_U4_N33_m400", "hubbard", 3, 12, 400, t=1.0, U=4.0,
                             target_of_sites=_doped_11_12,
                             description="3-leg Hubbard ladder 3x12, t=1, U=4, 33 electrons (17 up, 16 down), m=400")
HEISENBERG_4X16_M1000 = Workload("heisenberg_4x16_m1000", "heisenberg", 4, 16, 1000, J=1.0,
                                 target_of_sites=_sz_zero(4),
                                 description="4-leg Heisenberg ladder 4x16, J=1, S_z=0, m=1000")

# the single-superblock workloads by name
WORKLOADS = {w.name: w for w in (HEISENBERG_2X6_M16, HUBBARD_2X16_M256, HUBBARD_3X12_M400, HEISENBERG_4X16_M1000)}

# the benchmark set in its fixed order (the benchmark's --config index 1..5;
# 5 is the batch of 64 uneven superblocks)
BENCH_SET = (HEISENBERG_2X6_M16.name, HUBBARD_2X16_M256.name, HUBBARD_3X12_M400.name,
             HEISENBERG_4X16_M1000.name, "batch64")


def batch64(length: int | None = None):
    """The 64 uneven superblocks of the batch workload on ``length`` columns
    (default ``BATCH_LENGTH``)."""
    return _batch64_problems(BATCH_LENGTH if length is None else length)


def block_path(name: str) -> str:
    return os.path.join(BLOCK_DIR, f"{name}.npz")


def load_blocks(name: str):
    """Raw arrays of a frozen block file: ``{"L": {...}, "R": {...}}``."""
    with np.load(block_path(name), allow_pickle=False) as z:
        out = {"L": {}, "R": {}}
        for k in z.files:
            side, key = k[0], k[2:]
            out[side][key] = z[k]
    return out


def block_file_hash(name: str) -> str:
    h = hashlib.sha256()
    with open(block_path(name), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) vector (the start vectors and the Hv test vectors)."""
    return np.random.default_rng(seed).standard_normal(n)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """Outputs 0..n-1 of the SplitMix64 stream seeded with ``seed`` (Steele,
    Lea and Flood 2014): output c is mix(seed + (c+1) * 0x9E3779B97F4A7C15)."""
    c = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def splitmix_normal(n: int, seed: int) -> np.ndarray:
    """The library's seeded start vector: element i is the Box-Muller normal
    sqrt(-2 ln u1) cos(2 pi u2) of u = (out >> 11 + 1/2) 2^-53 for SplitMix64
    outputs 2i and 2i+1."""
    u = ((splitmix64(seed, 2 * n) >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u[0::2])) * np.cos(2.0 * np.pi * u[1::2])


def unit_vector(n: int, seed: int) -> np.ndarray:
    v = random_vector(n, seed)
    return v / math.sqrt(float(v @ v))
