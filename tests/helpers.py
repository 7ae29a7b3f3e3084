"""Shared set-up for the tests: build the same superblock on both sides.

The oracle side and the HIP side read the same frozen blocks and seeded
vectors from ``workloads``; nothing else is shared.
"""
from __future__ import annotations

import json
import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def reference_energy(name: str) -> float:
    with open(os.path.join(GOLDEN, "reference_energies.json")) as f:
        return float(json.load(f)[name]["E0"])


def oracle_superblock(wl: W.Workload, target=None):
    from oracle.blockio import block_from_arrays
    from oracle.superblock import Superblock
    raw = W.load_blocks(wl.name)
    return Superblock(block_from_arrays(raw["L"]), block_from_arrays(raw["R"]),
                      wl.target if target is None else target)


class GpuProblem:
    """Blocks and superblock of a workload on the device (HIP library)."""

    def __init__(self, ctx, wl: W.Workload, target=None, prec_mask=3):
        from paper_0707_0159_amd import d2d
        self.d2d = d2d
        raw = W.load_blocks(wl.name)
        self.model = d2d.make_model(wl.kind, wl.legs, wl.t, wl.U, wl.J)
        self.b1 = d2d.d2d_block_import(ctx, self.model, raw["L"])
        self.b4 = d2d.d2d_block_import(ctx, self.model, raw["R"])
        self.sb = d2d.d2d_sb_create(ctx, self.b1, self.b4, self.model,
                                    wl.target if target is None else target, prec_mask)
        self.info = d2d.d2d_sb_info(self.sb)

    def close(self):
        d = self.d2d
        d.d2d_sb_destroy(self.sb)
        d.d2d_block_destroy(self.b1)
        d.d2d_block_destroy(self.b4)


def rel_err(w, ref):
    w = np.asarray(w, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(w - ref) / np.linalg.norm(ref))
