"""Brute-force lattice Hamiltonians (test infrastructure).

The plain definition of the models the paper studies on an ``s``-leg x ``L``
ladder with open boundaries in both directions: the Heisenberg model with
J_z = J_xy and the Hubbard model with hopping ``-t`` and on-site ``+U``.
Site ``(x, y)`` (column ``x``, leg ``y``) has number ``x*s + y``; Hubbard mode
``2*site + sigma``.  A basis state is the product of creators in increasing
mode order acting on the vacuum, so ``c_a^dag c_b`` carries
``(-1)**(occupied modes strictly between a and b)``.

Built without any Kronecker product or block structure, so that it pins the
superblock construction from the outside.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp

from .local import popcount


def bonds(legs: int, length: int):
    """Nearest-neighbour bonds ``(site_a, site_b)`` with ``a < b``, OBC."""
    out = []
    for x in range(length):
        for y in range(legs):
            i = x * legs + y
            if y + 1 < legs:
                out.append((i, i + 1))
            if x + 1 < length:
                out.append((i, i + legs))
    return out


def _states_with_bits(positions, count):
    out = []
    for c in combinations(positions, count):
        s = 0
        for p in c:
            s |= 1 << p
        out.append(s)
    return np.array(sorted(out), dtype=np.int64)


def hubbard_basis(legs: int, length: int, nup: int, ndn: int) -> np.ndarray:
    ns = legs * length
    ups = _states_with_bits([2 * i for i in range(ns)], nup)
    dns = _states_with_bits([2 * i + 1 for i in range(ns)], ndn)
    return np.sort((ups[:, None] | dns[None, :]).reshape(-1))


def heisenberg_basis(legs: int, length: int, nup: int) -> np.ndarray:
    return _states_with_bits(list(range(legs * length)), nup)


def hubbard_hamiltonian(legs, length, t, U, nup, ndn):
    """Sparse Hubbard H on the ``(nup, ndn)`` sector; returns ``(H, basis)``."""
    basis = hubbard_basis(legs, length, nup, ndn)
    N = basis.size
    rows, cols, vals = [], [], []
    for a_site, b_site in bonds(legs, length):
        for s in range(2):
            a, b = 2 * a_site + s, 2 * b_site + s
            between = ((1 << b) - 1) ^ ((1 << (a + 1)) - 1)   # modes a < j < b
            for src_bit, dst_bit in ((b, a), (a, b)):          # c_dst^dag c_src
                mask = ((basis >> src_bit) & 1).astype(bool) & ~((basis >> dst_bit) & 1).astype(bool)
                src = basis[mask]
                dst = src ^ (1 << src_bit) ^ (1 << dst_bit)
                sign = np.where(popcount(src & between) % 2 == 0, 1.0, -1.0)
                rows.append(np.searchsorted(basis, dst))
                cols.append(np.nonzero(mask)[0])
                vals.append(-t * sign)
    double = np.zeros(N)
    for i in range(legs * length):
        double += ((basis >> (2 * i)) & 1) * ((basis >> (2 * i + 1)) & 1)
    rows.append(np.arange(N)); cols.append(np.arange(N)); vals.append(U * double)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return H, basis


def heisenberg_hamiltonian(legs, length, J, nup):
    """Sparse spin-1/2 Heisenberg H on the ``n_up`` sector; returns ``(H, basis)``."""
    basis = heisenberg_basis(legs, length, nup)
    N = basis.size
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    for a, b in bonds(legs, length):
        sa = ((basis >> a) & 1) - 0.5
        sb = ((basis >> b) & 1) - 0.5
        diag += J * sa * sb
        flip = sa != sb
        src = basis[flip]
        dst = src ^ (1 << a) ^ (1 << b)
        rows.append(np.searchsorted(basis, dst))
        cols.append(np.nonzero(flip)[0])
        vals.append(np.full(src.size, 0.5 * J))
    rows.append(np.arange(N)); cols.append(np.arange(N)); vals.append(diag)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    return H, basis


def lattice_hamiltonian(model, length, qn):
    """H of ``model`` on ``legs x length`` in sector ``qn = (n_up, n_dn)``."""
    if model.kind == "hubbard":
        return hubbard_hamiltonian(model.legs, length, model.t, model.U, qn[0], qn[1])
    return heisenberg_hamiltonian(model.legs, length, model.J, qn[0])


def ground_energy(H, k=1):
    """Lowest eigenvalue(s) of a sparse symmetric matrix (dense for small ones)."""
    N = H.shape[0]
    if N <= 3000:
        return np.linalg.eigvalsh(H.toarray())[:k]
    from scipy.sparse.linalg import eigsh
    return np.sort(eigsh(H, k=k, which="SA", tol=0, return_eigenvectors=False))
