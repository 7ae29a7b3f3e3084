"""Finite-system sweeps with the wavefunction transformation (test infrastructure).

TEST INFRASTRUCTURE ONLY (see the package header): the plain CPU version of
the sweeps whose ground-state energy the paper follows against the sweep
count (Fig. 3 and its discussion).  The paper states the result (convergence
within one or two sweeps) and not the procedure; this module takes the
standard finite-system algorithm for a superblock of two blocks and two
explicit columns (Fig. 1a), the reading recorded with the build's readings:

* Infinite phase: blocks grow from one column; the superblock of step k is
  left block (k columns) + two columns + right block (k columns), solved for
  the target of its 2k + 2 columns, and each enlarged half becomes the next
  block through its reduced density matrix (every block, truncated or not,
  is the enlarged half rotated onto its kept density-matrix eigenvectors;
  with m_keep at least the half's dimension the rotation keeps everything).
* Finite phase on L columns: the superblock at position l has the left
  block of l columns, columns l and l + 1, and the right block of the
  remaining L - l - 2 columns.  A step solves it, makes the new block of the
  half on the side the sweep moves to, and carries the ground state to the
  next position as the start vector (the wavefunction transformation):
  moving right, psi'[(i3, j1), (j3, j4)] = sum U_new[(i2, i1), j1]
  psi[(i2, i1), (i3, i4)] U_old[(j3, j4), i4], with U_new the kept
  eigenvectors that made the new left block and U_old the rotation that made
  the old right block from the next position's right half; moving left is
  the mirror image.
* The sweep turns at positions l_min and L - 2 - l_min, where the blocks
  stop having m states: blocks of fewer columns are exact (m = n^l_min), so
  the positions left out would change nothing.

Every block carries ``U``: its rotation from the enlarged half it was made
from (dense, half dimension x block states, half index = column state * m +
block state).
"""
from __future__ import annotations

import numpy as np

from .blocks import Block, column_block, left_half, right_half, truncate_half
from .dmrg import reduced_density_matrices
from .lanczos import lanczos_ground
from .local import Model, make_column
from .superblock import Superblock


def _grow(sb: Superblock, psi: np.ndarray, m_keep: int, side: str):
    """The block made from one enlarged half of ``sb`` by its reduced density
    matrix in the state ``psi``: ``(block with .U, truncation error)``; the
    block also records ``cut_gap``, the relative gap between the last kept
    and the first left-out density-matrix weight (1 when nothing is left out):
    a truncation is well defined only when it is not zero."""
    rhoL, rhoR, rows_of, cols_of = reduced_density_matrices(sb, psi)
    if side == "L":
        blk, _, trunc, spec, U = truncate_half(sb.left, rhoL, rows_of, m_keep)
    else:
        blk, _, trunc, spec, U = truncate_half(sb.right, rhoR, cols_of, m_keep)
    blk.U = np.asarray(U.todense())
    k = blk.dim
    blk.cut_gap = 1.0 if k >= spec.size or spec[k - 1] <= 0 else float((spec[k - 1] - spec[k]) / spec[k - 1])
    return blk, trunc


def _solve(sb: Superblock, v0, tol, res_tol=1e-12):
    """Ground state to a residual of ``res_tol * |E|``: the later blocks are
    made from this vector, so its accuracy (not only the energy's) carries
    into every later energy.  Lanczos restarted from its Ritz vector until
    the residual is met (at most 20 restarts)."""
    E, x, info = lanczos_ground(sb.hv_factored, v0, max_iter=600, tol=tol)
    its = info["iterations"]
    for _ in range(20):
        if info["residual"] <= res_tol * abs(E):
            break
        E, x, info = lanczos_ground(sb.hv_factored, x, max_iter=600, tol=tol)
        its += info["iterations"]
    return E, x, dict(info, iterations=its)


def wavefunction_transform(sb_from: Superblock, psi: np.ndarray, sb_to: Superblock, U_new: np.ndarray,
                           U_old: np.ndarray, direction: int) -> np.ndarray:
    """The state ``psi`` of ``sb_from`` carried to ``sb_to`` one column right
    (direction 0) or left (1); ``U_new`` is the rotation of the block made
    at this step, ``U_old`` that of the old block on the other side.  Full
    space, column-major V as the packed layout's index maps define it."""
    n, m, m2 = sb_from.n, sb_from.m, sb_to.m
    D, D2 = n * m, n * m2
    V = sb_from.unpack(psi).reshape(D, D, order="F")           # V[(i2, i1), (i3, i4)]
    if direction == 0:
        X = U_new.T @ V                                          # [j1, (i3, i4)]
        T = X.reshape(m2, m, n, order="F")                       # [j1, i4, i3]
        R = np.einsum("aki,ck->aic", T, U_old)                   # [j1, i3, (j3, j4)]
        W = R.reshape(D2, D2, order="F")                         # rows (i3, j1)
    else:
        Y = V @ U_new                                            # [(i2, i1), j4]
        Y3 = Y.reshape(m, n, m2, order="F")                      # [i1, i2, j4]
        R = np.einsum("rk,kib->rbi", U_old, Y3)                  # [(j2, j1), j4, i2]
        W = R.reshape(D2, D2, order="F")                         # columns (i2, j4)
    return sb_to.pack(W.reshape(-1, order="F"))


def infinite_blocks(model: Model, block_cols: int, m_keep: int, target_of_sites, tol=1e-13, seed=0):
    """Left and right blocks of 1 .. block_cols + 1 columns from the infinite
    phase, the last superblock (2 block_cols + 2 columns) and its ground state."""
    col = make_column(model)
    left, right = {1: column_block(col, "L")}, {1: column_block(col, "R")}
    left[1].U = None
    right[1].U = None
    sb, E, psi, hist = None, None, None, []
    for k in range(1, block_cols + 1):
        sb = Superblock(left[k], right[k], target_of_sites(model.legs * (2 * k + 2)))
        E, psi, _ = _solve(sb, np.random.default_rng(seed + k).standard_normal(sb.N), tol)
        left[k + 1], tl = _grow(sb, psi, m_keep, "L")
        right[k + 1], tr = _grow(sb, psi, m_keep, "R")
        hist.append(dict(block_cols=k, N=sb.N, energy=E, trunc_left=tl, trunc_right=tr,
                         cut_gap=min(left[k + 1].cut_gap, right[k + 1].cut_gap)))
    return left, right, sb, E, psi, hist


def sweep_positions(L: int, l_min: int, nsweeps: int):
    """``(position, direction)`` of every step: from the middle to the right
    turn, to the left turn, back to the middle, ``nsweeps`` times; direction
    0 moves the next position right, 1 left, -1 ends."""
    l0, l_max = L // 2 - 1, L - 2 - l_min
    steps = []
    for _ in range(nsweeps):
        steps += [(l, 0) for l in range(l0, l_max)]
        steps += [(l, 1) for l in range(l_max, l_min, -1)]
        steps += [(l, 0) for l in range(l_min, l0)]
    steps.append((l0, -1))
    return steps


def finite_sweeps(model: Model, L: int, m_keep: int, target_of_sites, l_min: int, nsweeps: int, tol=1e-13,
                  seed=0):
    """Energies along ``nsweeps`` finite-system sweeps on ``L`` columns.

    Returns a list of per-step records: position, direction, sweep index,
    superblock length, ground energy, the start vector's norm and energy
    (the transformed previous ground state; the first step starts from the
    infinite phase's state), the Lanczos products and the truncation error
    of the block made at the step."""
    if L % 2 or l_min < 1 or L - 2 - l_min <= l_min:
        raise ValueError("need an even L and 1 <= l_min < L/2 - 1")
    K = L // 2 - 1
    left, right, sb, _, psi, hist = infinite_blocks(model, K, m_keep, target_of_sites, tol=tol, seed=seed)
    inf_gap = min(h["cut_gap"] for h in hist)
    target = target_of_sites(model.legs * L)
    steps = sweep_positions(L, l_min, nsweeps)
    per_sweep = len(steps) // nsweeps if nsweeps else 1
    out = []
    # the infinite phase's last superblock is the finite phase's first (the
    # middle position): its ground state starts the sweeps
    guess = psi
    for s, (l, d) in enumerate(steps):
        g_norm = float(np.linalg.norm(guess))
        g_energy = float(guess @ sb.hv_factored(guess)) / g_norm ** 2
        E, psi, info = _solve(sb, guess, tol)
        rec = dict(step=s, sweep=s // per_sweep, position=l, direction=d, N=sb.N, energy=E,
                   guess_norm=g_norm, guess_energy=g_energy, products=info.get("iterations", 0),
                   infinite_cut_gap=inf_gap)
        if d == 0:
            newL, trunc = _grow(sb, psi, m_keep, "L")
            left[l + 1] = newL
            nxt = Superblock(newL, right[L - l - 3], target)
            guess = wavefunction_transform(sb, psi, nxt, newL.U, right[L - l - 2].U, 0)
            rec["cut_gap"] = newL.cut_gap
        elif d == 1:
            newR, trunc = _grow(sb, psi, m_keep, "R")
            right[L - l - 1] = newR
            nxt = Superblock(left[l - 1], newR, target)
            guess = wavefunction_transform(sb, psi, nxt, newR.U, left[l].U, 1)
            rec["cut_gap"] = newR.cut_gap
        else:
            trunc, nxt = 0.0, None
            rec["cut_gap"] = 1.0
        rec["trunc"] = trunc
        out.append(rec)
        sb = nxt
    return out
