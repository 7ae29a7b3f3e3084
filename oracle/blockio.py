"""Conversion between oracle blocks and the frozen block-file arrays
(test infrastructure).  The file layout is described in ``workloads``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .blocks import Block
from .local import Model

_KIND = {"heisenberg": 0, "hubbard": 1}
_KIND_NAME = {0: "heisenberg", 1: "hubbard"}


def _op_key(k):
    if k[0] == "c":
        return (0, k[1], k[2])
    if k[0] == "sz":
        return (1, k[1], 0)
    if k[0] == "sp":
        return (2, k[1], 0)
    raise ValueError(k)


def _key_of(row):
    a, y, s = (int(v) for v in row)
    return {0: ("c", y, s), 1: ("sz", y), 2: ("sp", y)}[a]


def block_to_arrays(B: Block) -> dict:
    secs = B.sectors()
    sec_qn = np.array([q for q, _, _ in secs], dtype=np.int64).reshape(-1, 2)
    sec_dim = np.array([b - a for _, a, b in secs], dtype=np.int64)
    H = sp.csr_matrix(B.H)
    Hparts = []
    for i, (q, a, b) in enumerate(secs):
        blk = H[a:b][:, a:b].toarray()
        # the Hamiltonian must not couple different sectors
        assert abs(H[a:b]).sum() - abs(blk).sum() < 1e-12 * max(1.0, abs(blk).sum())
        Hparts.append(blk.reshape(-1, order="F"))
    keys = sorted(B.edge, key=_op_key)
    op_key = np.array([_op_key(k) for k in keys], dtype=np.int64).reshape(-1, 3)
    op_blk, op_off, op_data = [], [], []
    off = 0
    for oi, k in enumerate(keys):
        O = sp.csr_matrix(B.edge[k])
        for sf, (_, a, b) in enumerate(secs):
            for st, (_, c, d) in enumerate(secs):
                blk = O[c:d][:, a:b]
                if blk.nnz == 0 or abs(blk).max() == 0.0:
                    continue
                dense = blk.toarray()
                op_blk.append((oi, sf, st))
                op_off.append(off)
                op_data.append(dense.reshape(-1, order="F"))
                off += dense.size
    cat = lambda parts: np.concatenate(parts) if parts else np.zeros(0)
    return {
        "kind": np.int64(_KIND[B.model.kind]), "legs": np.int64(B.model.legs),
        "ncols": np.int64(B.ncols), "side": np.int64(0 if B.side == "L" else 1),
        "t": np.float64(B.model.t), "U": np.float64(B.model.U), "J": np.float64(B.model.J),
        "sec_qn": sec_qn, "sec_dim": sec_dim, "H": cat(Hparts),
        "op_key": op_key, "op_blk": np.array(op_blk, dtype=np.int64).reshape(-1, 3),
        "op_off": np.array(op_off, dtype=np.int64), "op_data": cat(op_data),
    }


def block_from_arrays(a: dict) -> Block:
    model = Model(_KIND_NAME[int(a["kind"])], int(a["legs"]), t=float(a["t"]), U=float(a["U"]),
                  J=float(a["J"]))
    dims = np.asarray(a["sec_dim"], dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(dims)])
    m = int(starts[-1])
    qn = np.repeat(np.asarray(a["sec_qn"], dtype=np.int64).reshape(-1, 2), dims, axis=0)
    rows, cols, vals = [], [], []
    off = 0
    for i, d in enumerate(dims):
        blk = np.asarray(a["H"][off:off + d * d]).reshape(d, d, order="F")
        off += d * d
        r, c = np.meshgrid(np.arange(d), np.arange(d), indexing="ij")
        rows.append((r + starts[i]).ravel()); cols.append((c + starts[i]).ravel()); vals.append(blk.ravel())
    cat = lambda p: np.concatenate(p) if p else np.zeros(0)
    H = sp.csr_matrix((cat(vals), (cat(rows).astype(np.int64), cat(cols).astype(np.int64))), shape=(m, m))
    edge = {}
    keys = [_key_of(r) for r in np.asarray(a["op_key"]).reshape(-1, 3)]
    parts = {k: ([], [], []) for k in keys}
    for (oi, sf, st), o in zip(np.asarray(a["op_blk"]).reshape(-1, 3), np.asarray(a["op_off"])):
        df, dt = dims[sf], dims[st]
        blk = np.asarray(a["op_data"][o:o + df * dt]).reshape(dt, df, order="F")
        r, c = np.meshgrid(np.arange(dt), np.arange(df), indexing="ij")
        pr = parts[keys[oi]]
        pr[0].append((r + starts[st]).ravel()); pr[1].append((c + starts[sf]).ravel()); pr[2].append(blk.ravel())
    for k in keys:
        r, c, v = parts[k]
        edge[k] = sp.csr_matrix((cat(v), (cat(r).astype(np.int64), cat(c).astype(np.int64))), shape=(m, m))
    side = "L" if int(a["side"]) == 0 else "R"
    return Block(model, side, int(a["ncols"]), qn, H, edge, None)


def save_block_pair(path: str, L: Block, R: Block, meta: dict | None = None):
    out = {}
    for P, B in (("L_", L), ("R_", R)):
        for k, v in block_to_arrays(B).items():
            out[P + k] = v
    np.savez_compressed(path, **out)
