"""Infinite-system growth of blocks 1 and 4 (test infrastructure).

Fig. 1a: the superblock is block 1 + two single columns + block 4.  One DMRG
step solves the superblock ground state, forms the reduced density matrix of
each enlarged half (DMF), diagonalises it sector by sector (DMD) and keeps
``m`` states; the enlarged halves then become the blocks of the next, two
columns longer, superblock.

Left and right blocks are truncated independently, each from its own reduced
density matrix of the same ground state:

* left:  ``rho_L[q_L] = V[q] V[q]^T``
* right: ``rho_R[q_R] = V[q]^T V[q]``

with ``V[q]`` the ``d_L x d_R`` block of the packed ground state.
"""
from __future__ import annotations

import numpy as np

from .blocks import Block, block_from_half, column_block, truncate_half
from .lanczos import ground_state, ground_state_arpack
from .local import Model, make_column
from .superblock import Superblock


def reduced_density_matrices(sb: Superblock, psi: np.ndarray):
    """``({q_L: rho_L}, {q_R: rho_R}, rows_of, cols_of)`` of a packed state."""
    rhoL, rhoR, rows_of, cols_of = {}, {}, {}, {}
    Q = tuple(int(v) for v in sb.Q)
    for q, r, c, o in sb.sectors:
        dL, dR = r.size, c.size
        V = psi[o:o + dL * dR].reshape(dR, dL).T
        qr = (Q[0] - q[0], Q[1] - q[1])
        rhoL[q] = V @ V.T
        rhoR[qr] = V.T @ V
        rows_of[q] = r
        cols_of[qr] = c
    return rhoL, rhoR, rows_of, cols_of


def solve(sb: Superblock, seed=0, tol=1e-13, big=2_000_000):
    """Ground state of a superblock in its target sector (mode F products)."""
    if sb.N <= big:
        return ground_state(sb.hv_factored, sb.N, seed=seed, tol=tol, max_iter=600)
    v0 = np.random.default_rng(seed).standard_normal(sb.N)
    return ground_state_arpack(sb.hv_factored, sb.N, v0=v0, ncv=24, tol=tol)


def dmrg_step(L: Block, R: Block, target, m_keep: int, seed=0, tol=1e-12, log=None):
    """One infinite-system step; returns ``(E0, new_left, new_right, info)``."""
    sb = Superblock(L, R, target)
    E, psi, info = solve(sb, seed=seed, tol=tol)
    rhoL, rhoR, rows_of, cols_of = reduced_density_matrices(sb, psi)
    if sb.left.dim <= m_keep:
        newL = block_from_half(sb.left)
        tL = 0.0
    else:
        newL, _, tL, _, _ = truncate_half(sb.left, rhoL, rows_of, m_keep)
    if sb.right.dim <= m_keep:
        newR = block_from_half(sb.right)
        tR = 0.0
    else:
        newR, _, tR, _, _ = truncate_half(sb.right, rhoR, cols_of, m_keep)
    info = dict(info, N=sb.N, trunc_left=tL, trunc_right=tR, energy=E)
    if log is not None:
        log(info)
    return E, newL, newR, info


def infinite_system(model: Model, block_cols: int, m_keep: int, target_of_sites, seed=0,
                    tol=1e-12, log=None):
    """Grow blocks from one column to ``block_cols`` columns.

    ``target_of_sites(nsites)`` gives the target ``(n_up, n_dn)`` of the
    superblock with ``nsites`` sites at every intermediate length.
    Returns ``(left_block, right_block, history)``.
    """
    col = make_column(model)
    L = column_block(col, "L")
    R = column_block(col, "R")
    hist = []
    for k in range(1, block_cols):
        nsites = model.legs * (2 * k + 2)
        E, L, R, info = dmrg_step(L, R, target_of_sites(nsites), m_keep, seed=seed, tol=tol, log=log)
        info["block_cols"] = k
        hist.append(info)
    return L, R, hist
