"""Blocks of the direct 2-D DMRG (test infrastructure).

A block is a set of whole columns (Fig. 1a): "block 1" grows to the right,
"block 4" grows to the left, one column per DMRG step.  A block is stored as
explicit sparse matrices over its ``m`` states:

* ``H``     -- the block Hamiltonian (all bonds inside the block),
* ``edge``  -- the operators of the sites of the block's edge column, the one
               that faces the neighbouring column (rightmost column for a left
               block, leftmost for a right block).  Same keys as
               ``Column.ops``.  For fermions each annihilator carries the
               Jordan-Wigner string over the block's own modes that come before
               it (mode order: columns left to right, inside a column leg by
               leg, up before down).
* ``qn``    -- ``(n_up, n_dn)`` of every state; states are sorted by it
               (lexicographically, stable), so every sector is a contiguous
               range.
* ``occ``   -- for exact (untruncated) blocks only: the occupation bits of
               every state over the block's modes, column 0 of the block in
               the lowest bits.  Used to compare with the brute-force lattice.

Growth of the enlarged halves of the superblock (Eq. (1)):

* left half  ``block1 (x) column2``  with index ``i2*m + i1`` (the paper's
  ``(i2-1)m + i1``, column slow, block fast): matrix of ``O_1 (x) O_2`` is
  ``kron(O_2, O_1)``;
* right half ``column3 (x) block4``  with index ``i3*m + i4`` (the paper's
  ``(i3-1)m + i4``): matrix of ``O_3 (x) O_4`` is ``kron(O_3, O_4)``.

Truncation keeps the ``m`` eigenvectors of the reduced density matrix with the
largest eigenvalues (the DMF/DMD routines of the paper's performance
section).  Ties are broken by (sector ascending, index in sector ascending).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp

from .local import Column, Model, bond_terms, make_column


@dataclass
class Block:
    model: Model
    side: str                  # "L" (block 1) or "R" (block 4)
    ncols: int
    qn: np.ndarray             # (m, 2) int64, sorted lexicographically
    H: sp.csr_matrix
    edge: dict
    occ: Optional[np.ndarray] = None

    @property
    def dim(self) -> int:
        return self.qn.shape[0]

    @property
    def parity(self) -> np.ndarray:
        return np.where((self.qn.sum(axis=1) % 2) == 0, 1.0, -1.0)

    def sectors(self):
        """List of ``(qn tuple, start, stop)`` of the contiguous sector ranges."""
        out = []
        start = 0
        for i in range(1, self.dim + 1):
            if i == self.dim or tuple(self.qn[i]) != tuple(self.qn[start]):
                out.append((tuple(int(v) for v in self.qn[start]), start, i))
                start = i
        return out


def bits_per_column(model: Model) -> int:
    return 2 * model.legs if model.fermionic else model.legs


@dataclass
class Half:
    """An enlarged half (block (x) column or column (x) block), unsorted."""

    model: Model
    side: str
    ncols: int
    qn: np.ndarray
    H: sp.csr_matrix
    edge: dict               # operators of the new column, in the half's basis
    occ: Optional[np.ndarray] = None

    @property
    def dim(self) -> int:
        return self.qn.shape[0]


def column_block(col: Column, side: str) -> Block:
    """A block made of one exact column; its edge column is the column itself."""
    order = np.lexsort((np.arange(col.dim), col.qn[:, 1], col.qn[:, 0]))
    P = sp.csr_matrix((np.ones(col.dim), (np.arange(col.dim), order)), shape=(col.dim, col.dim))
    edge = {k: sp.csr_matrix(P @ v @ P.T) for k, v in col.ops.items()}
    return Block(col.model, side, 1, col.qn[order].copy(), sp.csr_matrix(P @ col.H @ P.T), edge,
                 occ=np.arange(col.dim, dtype=np.int64)[order])


def left_half(L: Block, col: Column) -> Half:
    """``block1 (x) column2`` on index ``i2*m + i1`` (Eq. (1), H_l)."""
    m, n = L.dim, col.dim
    Im, In = sp.identity(m, format="csr"), sp.identity(n, format="csr")
    H = sp.kron(In, L.H) + sp.kron(col.H, Im)
    for coef, A, B in bond_terms(L.model, L.edge, L.parity, col.ops):
        H = H + coef * sp.kron(B, A)
    qn = (col.qn[:, None, :] + L.qn[None, :, :]).reshape(m * n, 2)
    if L.model.fermionic:
        PL = sp.diags(L.parity).tocsr()
        edge = {k: sp.csr_matrix(sp.kron(v, PL)) for k, v in col.ops.items()}
    else:
        edge = {k: sp.csr_matrix(sp.kron(v, Im)) for k, v in col.ops.items()}
    occ = None
    if L.occ is not None:
        shift = L.ncols * bits_per_column(L.model)
        occ = (np.arange(n, dtype=np.int64)[:, None] << shift | L.occ[None, :]).reshape(-1)
    return Half(L.model, "L", L.ncols + 1, qn, sp.csr_matrix(H), edge, occ)


def right_half(col: Column, R: Block) -> Half:
    """``column3 (x) block4`` on index ``i3*m + i4`` (Eq. (1), H_r)."""
    m, n = R.dim, col.dim
    Im, In = sp.identity(m, format="csr"), sp.identity(n, format="csr")
    H = sp.kron(col.H, Im) + sp.kron(In, R.H)
    for coef, A, B in bond_terms(R.model, col.ops, col.parity, R.edge):
        H = H + coef * sp.kron(A, B)
    qn = (col.qn[:, None, :] + R.qn[None, :, :]).reshape(m * n, 2)
    # The new column holds the first modes of the enlarged block: no string.
    edge = {k: sp.csr_matrix(sp.kron(v, Im)) for k, v in col.ops.items()}
    occ = None
    if R.occ is not None:
        shift = bits_per_column(R.model)
        occ = (np.arange(n, dtype=np.int64)[:, None] | (R.occ[None, :] << shift)).reshape(-1)
    return Half(R.model, "R", R.ncols + 1, qn, sp.csr_matrix(H), edge, occ)


def block_from_half(h: Half) -> Block:
    """Exact block from an enlarged half: only a stable sort by quantum number."""
    order = np.lexsort((np.arange(h.dim), h.qn[:, 1], h.qn[:, 0]))
    P = sp.csr_matrix((np.ones(h.dim), (np.arange(h.dim), order)), shape=(h.dim, h.dim))
    edge = {k: sp.csr_matrix(P @ v @ P.T) for k, v in h.edge.items()}
    occ = None if h.occ is None else h.occ[order]
    return Block(h.model, h.side, h.ncols, h.qn[order].copy(), sp.csr_matrix(P @ h.H @ P.T), edge, occ)


def exact_block(model: Model, ncols: int, side: str) -> Block:
    """Exact block of ``ncols`` columns, grown by Kronecker products."""
    col = make_column(model)
    B = column_block(col, side)
    for _ in range(ncols - 1):
        B = block_from_half(left_half(B, col) if side == "L" else right_half(col, B))
    return B


def _fix_sign(vecs: np.ndarray) -> np.ndarray:
    idx = np.argmax(np.abs(vecs), axis=0)
    s = np.sign(vecs[idx, np.arange(vecs.shape[1])])
    s[s == 0] = 1.0
    return vecs * s


def truncate_half(h: Half, rho_blocks: dict, rows_of: dict, m_keep: int):
    """Project an enlarged half onto the ``m_keep`` leading density-matrix states.

    ``rho_blocks[q]`` is the reduced density matrix on the half's sector ``q``,
    whose rows are the half's basis states ``rows_of[q]`` (ascending).
    Returns ``(block, kept eigenvalues, discarded weight, full spectrum)``.
    """
    cand = []
    eig = {}
    for q in sorted(rho_blocks):
        w, U = np.linalg.eigh(rho_blocks[q])
        w, U = w[::-1], _fix_sign(U[:, ::-1])
        eig[q] = (w, U)
        for i, val in enumerate(w):
            cand.append((-val, q, i))
    cand.sort()
    kept = cand[:m_keep]
    spectrum = np.array([-c[0] for c in cand])
    keep_by_q = {}
    for _, q, i in kept:
        keep_by_q.setdefault(q, []).append(i)
    cols, rows, vals, qn = [], [], [], []
    kept_w = []
    j = 0
    for q in sorted(keep_by_q):
        idx = sorted(keep_by_q[q])
        w, U = eig[q]
        r = np.asarray(rows_of[q])
        for i in idx:
            rows.append(r)
            cols.append(np.full(r.size, j))
            vals.append(U[:, i])
            qn.append(q)
            kept_w.append(w[i])
            j += 1
    Ufull = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(h.dim, j))
    UT = sp.csr_matrix(Ufull.T)
    H = sp.csr_matrix(UT @ h.H @ Ufull)
    edge = {k: sp.csr_matrix(UT @ v @ Ufull) for k, v in h.edge.items()}
    blk = Block(h.model, h.side, h.ncols, np.array(qn, dtype=np.int64).reshape(-1, 2), H, edge, None)
    trunc = float(max(0.0, 1.0 - np.sum(kept_w)))
    return blk, np.array(kept_w), trunc, spectrum, Ufull
