"""Finite-system sweeps on the device (the energy-versus-sweep study of Fig. 3).

A driver over the C calls: every product, solve, density matrix and
transformation runs in the library's kernels; this module only orders the
calls and keeps the blocks.

* Infinite phase: one-column blocks (d2d_block_exact), then for k = 1 .. L/2 - 1
  the superblock of two k-column blocks and two columns is solved for the
  target of its 2k + 2 columns (d2d_lanczos from the library's seeded start
  vector) and both enlarged halves become the next blocks
  (d2d_density_matrix_both, m_keep states).
* Finite phase on L columns, position l = the left block's columns: solve
  (started from the transformed state of the previous position), make the
  block on the side the sweep moves to, create the next superblock and carry
  the state there (d2d_wavefunction_transform).  The sweep turns at l_min and
  L - 2 - l_min: the superblock needs blocks of equal size, which the blocks
  have from l_min columns on (with m = n^l_min the blocks of fewer columns
  are exact, and the positions left out would change nothing).
"""
from __future__ import annotations

import time

import torch

from . import d2d


def sweep_schedule(L: int, l_min: int, nsweeps: int):
    """(position, direction) per step: middle -> right turn -> left turn ->
    middle, nsweeps times, then a last solve in the middle (direction -1);
    direction 0 moves right, 1 left."""
    mid, right_turn = L // 2 - 1, L - 2 - l_min
    out = []
    for _ in range(nsweeps):
        out.extend((p, 0) for p in range(mid, right_turn))
        out.extend((p, 1) for p in range(right_turn, l_min, -1))
        out.extend((p, 0) for p in range(l_min, mid))
    out.append((mid, -1))
    return out


def _guess_stats(sb, prec_hv, g, w):
    """Norm of a start vector and its energy <g|H|g>/<g|g> (FP64 product)."""
    d2d.d2d_hv(sb, prec_hv, g, w)
    gg = float(torch.dot(g, g))
    return gg ** 0.5, float(torch.dot(g, w)) / gg


def finite_sweeps(ctx, model, L: int, m_keep: int, target_of_sites, l_min: int, nsweeps: int, prec=d2d.D2D_FP32,
                  k_in: int = 48, tol_res: float = 1e-9, window: int = 3, seed: int = 1, compare_random=False,
                  log=None):
    """Sweeps on the device; returns (infinite-phase records, per-step records).

    A step's record: step, sweep, position, direction, N, energy, the start
    vector's norm and energy, the solve's products per precision and
    restarts, the truncation error of the block made, and wall times in ms
    (solve, density matrix with its three phases, transformation).  With
    compare_random, each position is also solved from the library's seeded
    random start vector first (hv_count_random, ms_solve_random): the work
    the transformed start vector saves."""
    if L % 2 or l_min < 1 or L - 2 - l_min <= l_min:
        raise ValueError("need an even L and 1 <= l_min < L/2 - 1")
    legs = model.legs
    s = ctx.stream
    mask = 3 | (1 << prec)
    opts = d2d.lanczos_opts(prec=prec, k_in=k_in, max_restarts=300, tol_res=tol_res, reorth_window=window,
                            seed=seed)
    blocks = []                                   # every block made, destroyed at the end
    left = {1: d2d.d2d_block_exact(ctx, model, 1, 0)}
    right = {1: d2d.d2d_block_exact(ctx, model, 1, 1)}
    blocks += [left[1], right[1]]
    K = L // 2 - 1
    inf_recs, recs = [], []
    sb = psi = None
    try:
        for k in range(1, K + 1):
            if sb is not None:
                d2d.d2d_sb_destroy(sb)
            sb = d2d.d2d_sb_create(ctx, left[k], right[k], model, target_of_sites(legs * (2 * k + 2)), mask)
            N = d2d.d2d_sb_info(sb)["n"]
            with torch.cuda.stream(s):
                psi = torch.zeros(N, dtype=torch.float64, device="cuda")
            st, e, stats = d2d.d2d_lanczos(sb, opts, None, psi)
            # both halves grow: one call, their eigensolves sharing the streams
            left[k + 1], right[k + 1], te, _ = d2d.d2d_density_matrix_both(sb, psi, m_keep)
            tl, tr = float(te[0]), float(te[1])
            blocks += [left[k + 1], right[k + 1]]
            inf_recs.append(dict(block_cols=k, N=N, energy=e, trunc_left=tl, trunc_right=tr,
                                 hv_count=list(stats["hv_count"]), status=st))
            if log:
                log(inf_recs[-1])
        # the last infinite superblock is the middle position of the finite phase
        target = target_of_sites(legs * L)
        steps = sweep_schedule(L, l_min, nsweeps)
        per = len(steps) // nsweeps if nsweeps else 1
        guess = psi
        N = d2d.d2d_sb_info(sb)["n"]
        for i, (l, d) in enumerate(steps):
            with torch.cuda.stream(s):
                w = torch.empty(N, dtype=torch.float64, device="cuda")
                psi = torch.zeros(N, dtype=torch.float64, device="cuda")
            g_norm, g_energy = _guess_stats(sb, d2d.D2D_FP64, guess, w)
            extra = {}
            if compare_random:
                s.synchronize()
                t0 = time.perf_counter()
                _, e_r, st_r = d2d.d2d_lanczos(sb, opts, None, psi)
                extra = dict(hv_count_random=list(st_r["hv_count"]), energy_random=e_r,
                             ms_solve_random=(time.perf_counter() - t0) * 1e3)
            s.synchronize()
            t0 = time.perf_counter()
            st, e, stats = d2d.d2d_lanczos(sb, opts, guess, psi)
            t_solve = (time.perf_counter() - t0) * 1e3
            rec = dict(step=i, sweep=i // per, position=l, direction=d, N=N, energy=e, guess_norm=g_norm,
                       guess_energy=g_energy, hv_count=list(stats["hv_count"]), restarts=stats["restarts"],
                       status=st, ms_solve=t_solve, **extra)
            if d in (0, 1):
                t0 = time.perf_counter()
                blk, trunc, _, ms = d2d.d2d_density_matrix_timed(sb, psi, d, m_keep)
                t_dm = (time.perf_counter() - t0) * 1e3
                blocks.append(blk)
                if d == 0:
                    left[l + 1] = blk
                    nxt = d2d.d2d_sb_create(ctx, blk, right[L - l - 3], model, target, mask)
                else:
                    right[L - l - 1] = blk
                    nxt = d2d.d2d_sb_create(ctx, left[l - 1], blk, model, target, mask)
                N = d2d.d2d_sb_info(nxt)["n"]
                with torch.cuda.stream(s):
                    guess = torch.empty(N, dtype=torch.float64, device="cuda")
                s.synchronize()
                t0 = time.perf_counter()
                d2d.d2d_wavefunction_transform(sb, psi, nxt, guess, d)
                t_wft = (time.perf_counter() - t0) * 1e3
                d2d.d2d_sb_destroy(sb)
                sb = nxt
                rec.update(trunc=trunc, ms_dm=t_dm, ms_dm_phases=list(ms), ms_transform=t_wft)
            else:
                rec.update(trunc=0.0)
            recs.append(rec)
            if log:
                log(rec)
    finally:
        s.synchronize()
        if sb is not None:
            d2d.d2d_sb_destroy(sb)
        for b in blocks:
            d2d.d2d_block_destroy(b)
    return inf_recs, recs
