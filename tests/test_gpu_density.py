"""Reduced density matrix and truncation (DMF/DMD) of the HIP library against the oracle.

Both sides get the same state psi (the GPU ground state).  Checked: the full
spectrum of rho and the truncation error; the kept block's sector structure and
its Hamiltonian spectrum per sector; and the ground energy of the next, two
columns longer, superblock built from the new blocks.
"""
import numpy as np
import pytest

import workloads as W
from helpers import GpuProblem, oracle_superblock

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_0707_0159_amd import d2d
    assert torch.cuda.is_available(), "GPU tests need a device"
    c = d2d.d2d_ctx_create(0)
    yield c
    torch.cuda.synchronize()
    d2d.d2d_ctx_destroy(c)


def ground_state(ctx, prob, seed):
    from paper_0707_0159_amd import d2d
    n = prob.info["n"]
    with torch.cuda.stream(ctx.stream):
        v0 = torch.as_tensor(W.random_vector(n, seed)).to("cuda")
        psi = torch.zeros_like(v0)
    ctx.stream.synchronize()
    st, e, _ = d2d.d2d_lanczos(prob.sb, d2d.lanczos_opts(prec=0, k_in=24, tol_res=1e-11), v0, psi)
    ctx.stream.synchronize()
    assert st == 0
    return psi


def gap_cut(spec, target):
    """Largest m <= target whose cut does not split a degenerate group."""
    for m in range(target, 1, -1):
        if spec[m - 1] - spec[m] > 1e-7 * max(spec[0], 1e-300):
            return m
    return target


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,target_m", [(W.HEISENBERG_2X6_M16.name, 40), (W.HUBBARD_2X16_M256.name, 300),
                                           (W.HUBBARD_3X12_M400.name, 400), (W.HEISENBERG_4X16_M1000.name, 1000)])
def test_density_matrix_and_next_block(ctx, name, target_m):
    from oracle.blockio import block_from_arrays
    from oracle.blocks import truncate_half
    from oracle.dmrg import reduced_density_matrices
    from oracle.superblock import Superblock
    from paper_0707_0159_amd import d2d

    wl = W.WORKLOADS[name]
    prob = GpuProblem(ctx, wl)
    osb = oracle_superblock(wl)
    psi = ground_state(ctx, prob, wl.seed)
    psi_h = psi.cpu().numpy()
    rhoL, rhoR, rows_of, cols_of = reduced_density_matrices(osb, psi_h)
    spec_o = np.sort(np.concatenate([np.linalg.eigvalsh(r) for r in rhoL.values()]))[::-1]
    m_keep = gap_cut(spec_o, min(target_m, spec_o.size - 1))
    blocks = {}
    for side, rho, idx, half in ((0, rhoL, rows_of, osb.left), (1, rhoR, cols_of, osb.right)):
        blk, te, spec, ms = d2d.d2d_density_matrix_timed(prob.sb, psi, side, m_keep, spectrum_cap=200000)
        print(f"{name} side {side} m_keep {m_keep}: formation {ms[0]:.2f} ms, diagonalisation {ms[1]:.2f} ms, "
              f"renormalisation {ms[2]:.2f} ms", flush=True)
        ob, kept_w, te_o, spec_or, _ = truncate_half(half, rho, idx, m_keep)
        assert spec.size == spec_or.size
        assert np.max(np.abs(spec - spec_or)) <= 1e-12
        assert abs(te - te_o) <= 1e-12
        gb = block_from_arrays(dict(d2d.d2d_block_export(blk), kind=np.int64(prob.model.kind),
                                    legs=np.int64(wl.legs), ncols=np.int64(ob.ncols), side=np.int64(side),
                                    t=np.float64(wl.t), U=np.float64(wl.U), J=np.float64(wl.J)))
        assert gb.dim == ob.dim == m_keep
        assert np.array_equal(gb.qn, ob.qn)
        for (q, a, b), (q2, a2, b2) in zip(gb.sectors(), ob.sectors()):
            assert q == q2 and b - a == b2 - a2
            e1 = np.linalg.eigvalsh(gb.H[a:b][:, a:b].toarray())
            e2 = np.linalg.eigvalsh(ob.H[a:b][:, a:b].toarray())
            assert np.max(np.abs(e1 - e2)) <= 1e-10 * max(1.0, np.abs(e2).max())
        for k in ob.edge:
            n1 = np.linalg.norm(gb.edge[k].toarray())
            n2 = np.linalg.norm(ob.edge[k].toarray())
            assert abs(n1 - n2) <= 1e-10 * max(1.0, n2)
        blocks[side] = (gb, ob)
        d2d.d2d_block_destroy(blk)
    # next superblock (two more columns): same ground energy from either pair of blocks
    Q2 = wl.target_of_sites(wl.legs * (wl.length + 2))
    e_gpu = np.linalg.eigvalsh(Superblock(blocks[0][0], blocks[1][0], Q2).explicit().toarray())[0] \
        if name == W.HEISENBERG_2X6_M16.name else None
    if name == W.HEISENBERG_2X6_M16.name:
        e_or = np.linalg.eigvalsh(Superblock(blocks[0][1], blocks[1][1], Q2).explicit().toarray())[0]
        assert abs(e_gpu - e_or) <= 1e-10 * abs(e_or)
    prob.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", [W.HUBBARD_2X16_M256.name, W.HEISENBERG_4X16_M1000.name])
def test_both_halves_equal_two_calls(ctx, name):
    """d2d_density_matrix_both gives both halves' blocks and truncation errors
    bit for bit as two d2d_density_matrix calls (the eigensolves of the two
    halves share the streams; each sector's is the same computation)."""
    from paper_0707_0159_amd import d2d
    wl = W.WORKLOADS[name]
    prob = GpuProblem(ctx, wl)
    psi = ground_state(ctx, prob, wl.seed)
    single = []
    for side in (0, 1):
        blk, te, _ = d2d.d2d_density_matrix(prob.sb, psi, side, wl.m)
        single.append((d2d.d2d_block_export(blk), te))
        d2d.d2d_block_destroy(blk)
    with pytest.raises(RuntimeError):
        d2d.d2d_density_matrix_both(prob.sb, psi, 0)      # m_keep < 1: D2D_EINVAL, no block made
    bl, br, te2, ms = d2d.d2d_density_matrix_both(prob.sb, psi, wl.m)
    print(f"{name}: both halves in {ms[0]:.2f} + {ms[1]:.2f} + {ms[2]:.2f} ms")
    for side, blk in ((0, bl), (1, br)):
        ex = d2d.d2d_block_export(blk)
        ref, te = single[side]
        assert te2[side] == te
        assert set(ex) == set(ref)
        for k in ref:
            assert np.array_equal(np.asarray(ex[k]), np.asarray(ref[k])), (side, k)
        d2d.d2d_block_destroy(blk)
    prob.close()
