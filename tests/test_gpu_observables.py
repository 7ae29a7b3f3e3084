"""Local densities of Eqs. (2)-(4) on the explicit columns (d2d_column_densities).

* Against the oracle's sums over the same device state, element by element:
  both are float64 sums of the N weights psi^2 (which add up to 1) in
  different orders, so they agree to 2 N u (u = 2^-53).
* With exact blocks (the 2x6 Heisenberg ladder of m = 16, a 2x4 Hubbard
  ladder from d2d_block_exact) the ground state is the lattice's, so the
  densities equal the brute-force lattice ground state's on those columns,
  and Lieb-Mattis holds: s(x, y) = 0 for the singlet ground state.
* On the truncated 2x16 Hubbard ladder (m = 256) the staggered spin density
  S(x) of the centre columns is reported.
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


def _ground(ctx, sb, n, tol=1e-11):
    from paper_0707_0159_amd import d2d
    with torch.cuda.stream(ctx.stream):
        psi = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.stream.synchronize()
    st, e, _ = d2d.d2d_lanczos(sb, d2d.lanczos_opts(prec=d2d.D2D_FP64, k_in=32, tol_res=tol), None, psi)
    assert st == 0
    ctx.stream.synchronize()
    return e, psi


def _lattice_ground_densities(model, length, Q):
    from scipy.sparse.linalg import eigsh
    from oracle.lattice import lattice_hamiltonian
    from oracle.observables import lattice_densities
    H, basis = lattice_hamiltonian(model, length, Q)
    w, v = eigsh(H, k=2, which="SA", tol=1e-14, v0=np.ones(H.shape[0]))
    o = np.argsort(w)
    assert w[o[1]] - w[o[0]] > 1e-8
    return lattice_densities(model, length, basis, v[:, o[0]])


def test_heisenberg_2x6_exact_blocks(ctx):
    from oracle.local import Model
    from oracle.observables import column_densities, hole_and_spin_density
    from paper_0707_0159_amd import d2d
    wl = W.HEISENBERG_2X6_M16
    osb = oracle_superblock(wl)
    prob = GpuProblem(ctx, wl)
    try:
        _, psi = _ground(ctx, prob.sb, prob.info["n"])
        n_gpu = d2d.d2d_column_densities(prob.sb, psi, wl.legs)
        n_orc = column_densities(osb, psi.cpu().numpy())
        assert np.abs(n_gpu - n_orc).max() <= 2 * prob.info["n"] * 2.0 ** -53
        n_lat = _lattice_ground_densities(Model("heisenberg", 2, J=1.0), 6, wl.target)
        x2 = osb.L.ncols
        assert np.abs(n_gpu - n_lat[x2:x2 + 2]).max() <= 1e-8
        _, s = hole_and_spin_density(n_gpu)
        print("2x6 Heisenberg s(x, y):", s)
        assert np.abs(s).max() <= 1e-8          # Lieb-Mattis: singlet ground state
    finally:
        prob.close()


def test_hubbard_2x4_exact_blocks_from_the_library(ctx):
    from oracle.local import Model
    from oracle.observables import hole_and_spin_density
    from paper_0707_0159_amd import d2d
    model = d2d.make_model("hubbard", 2, 1.0, 6.0, 1.0)
    b1 = d2d.d2d_block_exact(ctx, model, 1, 0)
    b4 = d2d.d2d_block_exact(ctx, model, 1, 1)
    sb = d2d.d2d_sb_create(ctx, b1, b4, model, (4, 4), 3)
    try:
        n = d2d.d2d_sb_info(sb)["n"]
        _, psi = _ground(ctx, sb, n)
        n_gpu = d2d.d2d_column_densities(sb, psi, 2)
        n_lat = _lattice_ground_densities(Model("hubbard", 2, t=1.0, U=6.0), 4, (4, 4))
        assert np.abs(n_gpu - n_lat[1:3]).max() <= 1e-8
        h, s = hole_and_spin_density(n_gpu)
        print("2x4 Hubbard h:", h, "s:", s)
        assert np.abs(s).max() <= 1e-8
        # half filling and reflection symmetry of the open ladder: the two
        # centre columns carry the same density
        assert np.abs(h[0] - h[1]).max() <= 1e-8
    finally:
        d2d.d2d_sb_destroy(sb)
        d2d.d2d_block_destroy(b1)
        d2d.d2d_block_destroy(b4)


def test_hubbard_2x16_truncated_against_oracle(ctx):
    from oracle.observables import column_densities, hole_and_spin_density, staggered_max
    from paper_0707_0159_amd import d2d
    wl = W.HUBBARD_2X16_M256
    osb = oracle_superblock(wl)
    prob = GpuProblem(ctx, wl)
    try:
        _, psi = _ground(ctx, prob.sb, prob.info["n"], tol=1e-9)
        n_gpu = d2d.d2d_column_densities(prob.sb, psi, wl.legs)
        n_orc = column_densities(osb, psi.cpu().numpy())
        assert np.abs(n_gpu - n_orc).max() <= 2 * prob.info["n"] * 2.0 ** -53
        h, s = hole_and_spin_density(n_gpu)
        print(f"2x16 Hubbard m=256 centre columns: h {h}, S(x) {staggered_max(s)}")
        assert np.all(np.abs(h) <= 1.0) and np.all(np.abs(s) <= 1.0)
    finally:
        prob.close()
