"""One column of the ladder as explicit sparse matrices (test infrastructure).

A column is one rung of ``s`` sites ("block 2" and "block 3" of the
superblock, Fig. 2).  Its dimension is 4**s for the Hubbard model and 2**s for
the spin-1/2 Heisenberg model, which is where the 16^s m^2 / 4^s m^2 state
count of the introduction comes from.

Basis: integers ``b`` in ``range(dim)``.

* Hubbard: mode ``j = 2*y + sigma`` (leg ``y``, ``sigma`` 0 = up, 1 = down) is
  occupied when bit ``j`` of ``b`` is set.  The state is the product of
  creators taken in increasing mode order acting on the vacuum, so an
  annihilator of mode ``j`` picks up ``(-1)**(occupied modes below j)``.
* Heisenberg: bit ``y`` set means spin up on leg ``y``.

Model conventions (the paper gives only U/t and the fermion numbers): hopping
``-t`` on every nearest-neighbour bond, ``+U n_up n_dn`` on every site, no
chemical potential; spin model ``J (S^z S^z + (S^+ S^- + S^- S^+)/2)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


def popcount(x):
    x = np.asarray(x, dtype=np.int64)
    c = np.zeros_like(x)
    y = x.copy()
    while np.any(y):
        c += y & 1
        y >>= 1
    return c


@dataclass
class Model:
    """Model parameters.  ``kind`` is ``"heisenberg"`` or ``"hubbard"``."""

    kind: str
    legs: int
    t: float = 1.0
    U: float = 0.0
    J: float = 1.0

    @property
    def fermionic(self) -> bool:
        return self.kind == "hubbard"


@dataclass
class Column:
    """Explicit matrices of one column.

    ``ops`` holds the site operators that enter bonds:
      Hubbard:    ``ops[("c", y, sigma)]``   annihilator with in-column string
      Heisenberg: ``ops[("sz", y)]``, ``ops[("sp", y)]``
    """

    model: Model
    dim: int
    qn: np.ndarray            # (dim, 2) int64: (n_up, n_dn)
    H: sp.csr_matrix          # rung bonds (+ on-site U)
    ops: dict = field(default_factory=dict)

    @property
    def parity(self) -> np.ndarray:
        return np.where((self.qn.sum(axis=1) % 2) == 0, 1.0, -1.0)


def _annihilator(dim: int, j: int) -> sp.csr_matrix:
    b = np.arange(dim, dtype=np.int64)
    occ = (b >> j) & 1
    src = b[occ == 1]
    sign = np.where(popcount(src & ((1 << j) - 1)) % 2 == 0, 1.0, -1.0)
    dst = src ^ (1 << j)
    return sp.csr_matrix((sign, (dst, src)), shape=(dim, dim))


def _spin_ops(dim: int, y: int):
    b = np.arange(dim, dtype=np.int64)
    up = (b >> y) & 1
    sz = sp.diags(up - 0.5).tocsr()
    src = b[up == 0]
    splus = sp.csr_matrix((np.ones(src.size), (src | (1 << y), src)), shape=(dim, dim))
    return sz, splus


def hubbard_column(legs: int, t: float, U: float) -> Column:
    model = Model("hubbard", legs, t=t, U=U)
    dim = 4 ** legs
    b = np.arange(dim, dtype=np.int64)
    nup = sum(((b >> (2 * y)) & 1) for y in range(legs))
    ndn = sum(((b >> (2 * y + 1)) & 1) for y in range(legs))
    qn = np.stack([nup, ndn], axis=1).astype(np.int64)
    ops = {}
    for y in range(legs):
        for s in range(2):
            ops[("c", y, s)] = _annihilator(dim, 2 * y + s)
    H = sp.csr_matrix((dim, dim))
    for y in range(legs - 1):
        for s in range(2):
            a, c = ops[("c", y, s)], ops[("c", y + 1, s)]
            H = H - t * (a.T @ c + c.T @ a)
    for y in range(legs):
        nu = ops[("c", y, 0)].T @ ops[("c", y, 0)]
        nd = ops[("c", y, 1)].T @ ops[("c", y, 1)]
        H = H + U * (nu @ nd)
    return Column(model, dim, qn, sp.csr_matrix(H), ops)


def heisenberg_column(legs: int, J: float) -> Column:
    model = Model("heisenberg", legs, J=J)
    dim = 2 ** legs
    b = np.arange(dim, dtype=np.int64)
    nup = popcount(b)
    qn = np.stack([nup, np.zeros_like(nup)], axis=1).astype(np.int64)
    ops = {}
    for y in range(legs):
        sz, splus = _spin_ops(dim, y)
        ops[("sz", y)] = sz
        ops[("sp", y)] = splus
    H = sp.csr_matrix((dim, dim))
    for y in range(legs - 1):
        H = H + J * (ops[("sz", y)] @ ops[("sz", y + 1)]
                     + 0.5 * (ops[("sp", y)] @ ops[("sp", y + 1)].T
                              + ops[("sp", y)].T @ ops[("sp", y + 1)]))
    return Column(model, dim, qn, sp.csr_matrix(H), ops)


def make_column(model: Model) -> Column:
    if model.kind == "hubbard":
        col = hubbard_column(model.legs, model.t, model.U)
    elif model.kind == "heisenberg":
        col = heisenberg_column(model.legs, model.J)
    else:
        raise ValueError(model.kind)
    col.model = model
    return col


def bond_terms(model: Model, ops_x: dict, parity_x: np.ndarray, ops_y: dict):
    """Leg bonds between part X (whose modes come first) and part Y.

    Returns ``[(coef, A, B), ...]`` meaning ``sum coef * (A on X) (x) (B on Y)``.
    ``ops_x`` / ``ops_y`` hold the operators of the sites that face each other
    (same leg ``y``).  For fermions the Jordan-Wigner string of X's modes is
    folded into the X factor: c_x^dag c_y = (c_x^dag P_X) (x) c_y and
    c_y^dag c_x = (P_X c_x) (x) c_y^dag, with P_X = (-1)^{N_X}.
    """
    terms = []
    if model.kind == "hubbard":
        P = sp.diags(parity_x).tocsr()
        for y in range(model.legs):
            for s in range(2):
                cx, cy = ops_x[("c", y, s)], ops_y[("c", y, s)]
                terms.append((-model.t, sp.csr_matrix(cx.T @ P), cy))
                terms.append((-model.t, sp.csr_matrix(P @ cx), sp.csr_matrix(cy.T)))
    else:
        for y in range(model.legs):
            szx, spx = ops_x[("sz", y)], ops_x[("sp", y)]
            szy, spy = ops_y[("sz", y)], ops_y[("sp", y)]
            terms.append((model.J, szx, szy))
            terms.append((0.5 * model.J, spx, sp.csr_matrix(spy.T)))
            terms.append((0.5 * model.J, sp.csr_matrix(spx.T), spy))
    return terms
