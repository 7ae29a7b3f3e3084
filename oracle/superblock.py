"""The four-block superblock Hamiltonian of Eq. (1) and its product with v
(test infrastructure).

Blocks, left to right: block 1 (``m`` states, index ``i1``), column 2 (``n``
states, ``i2``), column 3 (``i3``), block 4 (``i4``).  Eq. (1) splits H into

* ``H_l`` on ``(i1, i2)``: block 1, column 2 and the bonds between them,
* ``H_r`` on ``(i3, i4)``: column 3, block 4 and the bonds between them,
* ``H_c`` on ``(i2, i3)``: only the leg bonds between columns 2 and 3
  (the intra-column terms already sit in H_l and H_r; counting them again in
  H_c would double them).

Index maps (0-based forms of the paper's 1-based ones):

* vector:  ``idx = i3*m*m*n + i4*m*n + i2*m + i1``
* ``V``    (``mn x nm``): row ``i2*m + i1``, column ``i3*m + i4``
  => ``V = reshape(v, (mn, mn), order="F")``
* ``V_c``  (``n^2 x m^2``): row ``i3*n + i2``, column ``i4*m + i1``.

The paper turns the three products into ``H_l V``, ``V H_r^T`` and
``H_c V_c``.  Restricted to a target quantum number ``Q`` the superblock
vector is block sparse in ``(q_L, Q - q_L)``; it is stored *packed*: sector
pairs in ascending ``q_L`` (lexicographic ``(n_up, n_dn)``), each block
column-major ``d_L x d_R``, rows in ascending ``i2*m + i1``, columns in
ascending ``i3*m + i4``.

Two independent products:

* mode X (``hv_explicit``): one explicit sparse matrix
  ``kron(H_r, I) + kron(I, H_l) + Pi^T kron(I, H_c) Pi`` restricted to the
  target (small systems only);
* mode F (``hv_factored``): the paper's matrix form, sector by sector, with
  ``H_c V_c`` done on an explicit gather of V_c.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .blocks import Block, left_half, right_half, bits_per_column
from .local import Column, Model, bond_terms, make_column


class Superblock:
    def __init__(self, L: Block, R: Block, target, col: Column | None = None):
        if L.model.kind != R.model.kind or L.model.legs != R.model.legs:
            raise ValueError("blocks of different models")
        self.model: Model = L.model
        self.col = col if col is not None else make_column(self.model)
        self.L, self.R = L, R
        self.Q = np.asarray(target, dtype=np.int64).reshape(2)
        m1, m4, n = L.dim, R.dim, self.col.dim
        if m1 != m4:
            raise ValueError("the paper's index maps assume blocks 1 and 4 of equal size m")
        self.m, self.n = m1, n
        lh = left_half(L, self.col)
        rh = right_half(self.col, R)
        self.left, self.right = lh, rh
        self.H_l, self.H_r = lh.H, rh.H
        # H_c on index i3*n + i2: matrix of O_2 (x) O_3 is kron(O_3, O_2).
        Hc = sp.csr_matrix((n * n, n * n))
        for coef, A, B in bond_terms(self.model, self.col.ops, self.col.parity, self.col.ops):
            Hc = Hc + coef * sp.kron(B, A)
        self.H_c = sp.csr_matrix(Hc)
        self._layout()

    # ---------------------------------------------------------------- layout
    def _layout(self):
        qL, qR = self.left.qn, self.right.qn
        keyL = [tuple(q) for q in qL]
        keyR = [tuple(q) for q in qR]
        Q = tuple(int(v) for v in self.Q)
        rows_of, cols_of = {}, {}
        for i, k in enumerate(keyL):
            rows_of.setdefault(k, []).append(i)
        for i, k in enumerate(keyR):
            cols_of.setdefault(k, []).append(i)
        self.sectors = []      # (qL, rows, cols, offset)
        off = 0
        for q in sorted(rows_of):
            qr = (Q[0] - q[0], Q[1] - q[1])
            if qr not in cols_of:
                continue
            r = np.array(rows_of[q], dtype=np.int64)
            c = np.array(cols_of[qr], dtype=np.int64)
            self.sectors.append((q, r, c, off))
            off += r.size * c.size
        self.N = off
        mn = self.m * self.n
        self.sec_of_left = np.full(mn, -1, dtype=np.int64)
        self.row_pos = np.full(mn, -1, dtype=np.int64)
        self.col_pos = np.full(mn, -1, dtype=np.int64)
        for s, (q, r, c, o) in enumerate(self.sectors):
            self.sec_of_left[r] = s
            self.row_pos[r] = np.arange(r.size)
            self.col_pos[c] = np.arange(c.size)
        self.sec_dL = np.array([s[1].size for s in self.sectors], dtype=np.int64)
        self.sec_dR = np.array([s[2].size for s in self.sectors], dtype=np.int64)
        self.sec_off = np.array([s[3] for s in self.sectors], dtype=np.int64)
        self._dense = None
        self._central = None

    def full_index_of_packed(self) -> np.ndarray:
        """Paper's vector index (P: element ``(i3-1)m^2n + ...``) of every packed slot."""
        mn = self.m * self.n
        parts = []
        for q, r, c, o in self.sectors:
            parts.append((c[:, None] * mn + r[None, :]).reshape(-1))   # column-major block
        return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)

    def pack(self, v_full: np.ndarray) -> np.ndarray:
        return np.asarray(v_full)[self.full_index_of_packed()]

    def unpack(self, v: np.ndarray) -> np.ndarray:
        out = np.zeros((self.m * self.n) ** 2)
        out[self.full_index_of_packed()] = v
        return out

    def indices_of_packed(self):
        """``(i1, i2, i3, i4)`` of every packed slot (0-based)."""
        full = self.full_index_of_packed()
        m, n = self.m, self.n
        i1 = full % m
        i2 = (full // m) % n
        i4 = (full // (m * n)) % m
        i3 = full // (m * m * n)
        return i1, i2, i3, i4

    # ---------------------------------------------------------------- mode X
    def vc_index_of_full(self) -> np.ndarray:
        """Index of each full-vector slot in the column-major ``V_c``."""
        m, n = self.m, self.n
        idx = np.arange((m * n) ** 2, dtype=np.int64)
        i1 = idx % m
        i2 = (idx // m) % n
        i4 = (idx // (m * n)) % m
        i3 = idx // (m * m * n)
        return (i4 * m + i1) * (n * n) + i3 * n + i2

    def explicit(self, full_space: bool = False, absolute: bool = False) -> sp.csr_matrix:
        """H as one sparse matrix (mode X), on the target or the full space.

        With ``absolute`` the three parts enter with the absolute values of
        their entries, ``kron(|H_r|, I) + kron(I, |H_l|) + Pi^T kron(I, |H_c|) Pi``:
        the sum of the magnitudes of the terms that make up each element of
        ``H v`` (an upper bound of ``|H|`` entry by entry)."""
        m, n = self.m, self.n
        mn = m * n
        I_mn = sp.identity(mn, format="csr")
        fix = abs if absolute else (lambda a: a)
        H = sp.kron(fix(self.H_r), I_mn) + sp.kron(I_mn, fix(self.H_l))
        vc = self.vc_index_of_full()
        Hc_big = sp.csr_matrix(sp.kron(sp.identity(m * m, format="csr"), fix(self.H_c)))
        H = sp.csr_matrix(H + Hc_big[vc][:, vc])
        if full_space:
            return H
        sel = self.full_index_of_packed()
        return sp.csr_matrix(H[sel][:, sel])

    def hv_explicit(self, v: np.ndarray) -> np.ndarray:
        if getattr(self, "_Hx", None) is None:
            self._Hx = self.explicit()
        return self._Hx @ v

    # ---------------------------------------------------------------- mode F
    def dense_sectors(self, column_offdiagonal: bool = True):
        """``H_l`` and ``H_r`` restricted to each sector, as dense FP64 blocks.

        With ``column_offdiagonal=False``, without the explicit column's own
        off-diagonal terms (``1 (x) offdiag(h_col)`` on the half index
        ``column state * m + block state``): the part of each half that acts
        on the column alone and moves it to another state, which a product
        may apply as scaled copies of rectangles of ``V`` instead (the
        sectors' sum is unchanged: those terms conserve the column's quantum
        numbers)."""
        if column_offdiagonal:
            if self._dense is None:
                HL = sp.csr_matrix(self.H_l)
                HR = sp.csr_matrix(self.H_r)
                self._dense = [(HL[r][:, r].toarray(), HR[c][:, c].toarray()) for _, r, c, _ in self.sectors]
            return self._dense
        off = sp.csr_matrix(self.col.H) - sp.diags(sp.csr_matrix(self.col.H).diagonal())
        part = sp.csr_matrix(sp.kron(off, sp.identity(self.m, format="csr")))
        HL = sp.csr_matrix(self.H_l - part)
        HR = sp.csr_matrix(self.H_r - part)
        return [(HL[r][:, r].toarray(), HR[c][:, c].toarray()) for _, r, c, _ in self.sectors]

    def column_offdiagonal_part(self) -> sp.csr_matrix:
        """``1 (x) offdiag(h_col)`` on either half's index (the same matrix for
        both halves: column state slow, block state fast)."""
        off = sp.csr_matrix(self.col.H) - sp.diags(sp.csr_matrix(self.col.H).diagonal())
        return sp.csr_matrix(sp.kron(off, sp.identity(self.m, format="csr")))

    def central_groups(self):
        """Gather plan for ``H_c V_c``, one group per central sector.

        For a central pair of quantum number ``q23`` the columns of V_c that
        can be nonzero are the ``(i4, i1)`` with ``q1 + q4 = Q - q23``.  Each
        group holds ``(H_c restricted to q23, pidx)`` where ``pidx[row, col]``
        is the packed slot of ``V_c[row, col]``.
        """
        if self._central is not None:
            return self._central
        m, n = self.m, self.n
        qcol = self.col.qn
        q1, q4 = self.L.qn, self.R.qn
        # central index i3*n + i2 -> quantum number of the pair
        c_i3, c_i2 = np.divmod(np.arange(n * n), n)
        q23 = qcol[c_i3] + qcol[c_i2]
        # V_c column index i4*m + i1 -> quantum number of (i1, i4)
        v_i4, v_i1 = np.divmod(np.arange(m * m), m)
        q14 = q4[v_i4] + q1[v_i1]
        Hc = sp.csr_matrix(self.H_c)
        groups = []
        keys23 = {}
        for i, q in enumerate(map(tuple, q23)):
            keys23.setdefault(q, []).append(i)
        keys14 = {}
        for i, q in enumerate(map(tuple, q14)):
            keys14.setdefault(q, []).append(i)
        Q = tuple(int(v) for v in self.Q)
        for q, rows in sorted(keys23.items()):
            cq = (Q[0] - q[0], Q[1] - q[1])
            if cq not in keys14:
                continue
            rows = np.array(rows, dtype=np.int64)
            cols = np.array(keys14[cq], dtype=np.int64)
            i3, i2 = c_i3[rows], c_i2[rows]
            i4, i1 = v_i4[cols], v_i1[cols]
            Lidx = i2[:, None] * m + i1[None, :]
            Ridx = i3[:, None] * m + i4[None, :]
            s = self.sec_of_left[Lidx]
            if np.any(s < 0):
                raise AssertionError("central gather left the target space")
            pidx = self.sec_off[s] + self.col_pos[Ridx] * self.sec_dL[s] + self.row_pos[Lidx]
            groups.append((Hc[rows][:, rows].toarray(), pidx))
        self._central = groups
        return groups

    def hv_factored(self, v: np.ndarray) -> np.ndarray:
        """``w = H_l V + V H_r^T + unvec(H_c V_c)`` on the packed vector (mode F)."""
        v = np.asarray(v, dtype=np.float64)
        w = np.zeros_like(v)
        for (q, r, c, o), (hl, hr) in zip(self.sectors, self.dense_sectors()):
            dL, dR = r.size, c.size
            V = v[o:o + dL * dR].reshape(dR, dL).T
            W = hl @ V + V @ hr.T
            w[o:o + dL * dR] = W.T.reshape(-1)
        for hc, pidx in self.central_groups():
            w[pidx] += hc @ v[pidx]
        return w

    def hv_abs_bound(self, v: np.ndarray) -> np.ndarray:
        """``|H_l| |V| + |V| |H_r|^T + unvec(|H_c| |V_c|)`` of ``|v|`` (mode F on
        absolute values, packed).  Element i is the sum of the magnitudes of
        every product term that enters ``(H v)_i`` in the matrix form of Eq. (1),
        so any summation order of those terms in a precision with unit roundoff
        u errs by at most about (number of terms) * u times it."""
        a = np.abs(np.asarray(v, dtype=np.float64))
        w = np.zeros_like(a)
        for (q, r, c, o), (hl, hr) in zip(self.sectors, self.dense_sectors()):
            dL, dR = r.size, c.size
            V = a[o:o + dL * dR].reshape(dR, dL).T
            W = np.abs(hl) @ V + V @ np.abs(hr).T
            w[o:o + dL * dR] = W.T.reshape(-1)
        for hc, pidx in self.central_groups():
            w[pidx] += np.abs(hc) @ a[pidx]
        return w

    # ---------------------------------------------------------------- helpers
    def sector_table(self):
        """``[(qL, dL, dR, offset)]`` in packed order."""
        return [(q, r.size, c.size, o) for q, r, c, o in self.sectors]

    def occupation_of_packed(self) -> np.ndarray:
        """Occupation bits (lattice basis) of every packed slot; exact blocks only."""
        if self.L.occ is None or self.R.occ is None:
            raise ValueError("needs exact blocks")
        bpc = bits_per_column(self.model)
        i1, i2, i3, i4 = self.indices_of_packed()
        k1 = self.L.ncols
        return (self.L.occ[i1] | (i2.astype(np.int64) << (k1 * bpc))
                | (i3.astype(np.int64) << ((k1 + 1) * bpc))
                | (self.R.occ[i4] << ((k1 + 2) * bpc)))
