"""Pins of the oracle's block files, its element-wise bound, the parity
checker and the stored reference energies (CPU only).

* Block files (the frozen inputs both sides read): exact and truncated
  Heisenberg and Hubbard blocks come back from the file bit for bit; the
  file's operator blocks follow the documented layout, checked against the
  matrix elements of the edge-column operators written out from the
  occupation bits of exact blocks (Appendix A's Jordan-Wigner convention),
  independently of the reader; an exact-block superblock read back from the
  file equals the brute-force lattice Hamiltonian (fermion strings included).
* hv_abs_bound: mode F on absolute values equals the explicit mode X sum of
  absolute parts, and bounds |H v| and |H_lattice| |v| element by element.
* The element-wise checker fails a 1% error on one 16 x 16 tile of a small
  sector of the 4-leg m=1000 superblock, and on its smallest sector block,
  which the global 2-norm bar misses.
* Reference energies: stored residuals, the lattice-ED figure, and the
  Kato-Temple bracket of every reference that rests on one ARPACK run.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle.blockio as bio
import workloads as W
from oracle.blocks import exact_block
from oracle.dmrg import dmrg_step
from oracle.lattice import lattice_hamiltonian
from oracle.local import Model
from oracle.superblock import Superblock

from helpers import parity

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "reference_energies.json")


def _roundtrip(tmp_path, monkeypatch, L, R, name="rt"):
    monkeypatch.setattr(W, "BLOCK_DIR", str(tmp_path))
    bio.save_block_pair(W.block_path(name), L, R)
    raw = W.load_blocks(name)
    return bio.block_from_arrays(raw["L"]), bio.block_from_arrays(raw["R"]), raw


def _same_block(a, b):
    assert a.model == b.model and a.side == b.side and a.ncols == b.ncols
    assert np.array_equal(a.qn, b.qn)
    assert np.array_equal(sp.csr_matrix(a.H).toarray(), sp.csr_matrix(b.H).toarray())
    assert sorted(a.edge) == sorted(b.edge)
    for k in a.edge:
        assert np.array_equal(sp.csr_matrix(a.edge[k]).toarray(), sp.csr_matrix(b.edge[k]).toarray()), k


def _truncated_pair(model, Q, m_keep):
    """Blocks of two columns truncated to m_keep from a 4-column superblock's ground state."""
    _, L, R, _ = dmrg_step(exact_block(model, 1, "L"), exact_block(model, 1, "R"), Q, m_keep, tol=1e-12)
    return L, R


BLOCK_CASES = {
    "heisenberg_exact": lambda: (exact_block(Model("heisenberg", 2, J=1.0), 2, "L"),
                                 exact_block(Model("heisenberg", 2, J=1.0), 2, "R")),
    "hubbard_exact": lambda: (exact_block(Model("hubbard", 2, t=1.0, U=4.0), 1, "L"),
                              exact_block(Model("hubbard", 2, t=1.0, U=4.0), 1, "R")),
    "heisenberg_truncated": lambda: _truncated_pair(Model("heisenberg", 2, J=1.0), (4, 0), 10),
    "hubbard_truncated": lambda: _truncated_pair(Model("hubbard", 2, t=1.0, U=8.0), (4, 4), 40),
}


@pytest.mark.parametrize("case", sorted(BLOCK_CASES))
def test_block_file_roundtrip_bit_for_bit(tmp_path, monkeypatch, case):
    L, R = BLOCK_CASES[case]()
    L2, R2, _ = _roundtrip(tmp_path, monkeypatch, L, R)
    _same_block(L, L2)
    _same_block(R, R2)


def test_planted_transpose_in_the_writer_is_caught(tmp_path, monkeypatch):
    """Operator blocks written row-major instead of column-major (for a
    square block the transpose, which swaps S^+ and S^- and which no
    Heisenberg energy would show) do not come back."""
    L, R = BLOCK_CASES["heisenberg_truncated"]()
    orig = bio.block_to_arrays

    def transposed(B):
        a = orig(B)
        dims = a["sec_dim"]
        data = a["op_data"].copy()
        for (oi, sf, st), o in zip(a["op_blk"], a["op_off"]):
            df, dt = int(dims[sf]), int(dims[st])
            blk = data[o:o + df * dt].reshape(dt, df, order="F")
            data[o:o + df * dt] = blk.reshape(-1, order="C")      # row-major instead of column-major
        a["op_data"] = data
        return a

    monkeypatch.setattr(bio, "block_to_arrays", transposed)
    L2, R2, _ = _roundtrip(tmp_path, monkeypatch, L, R)
    with pytest.raises(AssertionError):
        _same_block(L, L2)


def _edge_matrix_from_bits(B, key):
    """<to|O|from> of an edge-column operator of an exact block, from the
    occupation bits alone: S^z, S^+ for spins; for fermions the annihilator
    with the sign (-1)^(occupied modes of the block before it), modes ordered
    columns left to right, inside a column leg by leg, up before down."""
    model, occ, m = B.model, B.occ, B.dim
    pos = {int(o): i for i, o in enumerate(occ)}
    M = np.zeros((m, m))
    edge_col = B.ncols - 1 if B.side == "L" else 0
    if model.kind == "heisenberg":
        y = key[1]
        bit = edge_col * model.legs + y
        for j, o in enumerate(occ):
            up = (int(o) >> bit) & 1
            if key[0] == "sz":
                M[j, j] = 0.5 if up else -0.5
            elif key[0] == "sp" and not up:
                M[pos[int(o) | (1 << bit)], j] = 1.0
        return M
    _, y, s = key
    bit = (edge_col * model.legs + y) * 2 + s
    for j, o in enumerate(occ):
        o = int(o)
        if (o >> bit) & 1:
            sign = -1.0 if bin(o & ((1 << bit) - 1)).count("1") % 2 else 1.0
            M[pos[o ^ (1 << bit)], j] = sign
    return M


@pytest.mark.parametrize("case", ["heisenberg_exact", "hubbard_exact"])
def test_block_file_layout_against_occupation_bits(tmp_path, monkeypatch, case):
    """The raw file arrays, read by the layout the header documents (per
    sector a column-major d x d Hamiltonian block; per operator block a
    column-major d_to x d_from block of (op index, sector from, sector to))
    without the oracle's reader, hold the edge operators that the occupation
    bits define."""
    L, R = BLOCK_CASES[case]()
    _, _, raw = _roundtrip(tmp_path, monkeypatch, L, R)
    for B, a in ((L, raw["L"]), (R, raw["R"])):
        dims = a["sec_dim"]
        starts = np.concatenate([[0], np.cumsum(dims)])
        m = int(starts[-1])
        keys = [tuple(int(x) for x in r) for r in a["op_key"]]
        ops = {k: np.zeros((m, m)) for k in keys}
        for (oi, sf, st), o in zip(a["op_blk"], a["op_off"]):
            df, dt = int(dims[sf]), int(dims[st])
            ops[keys[oi]][starts[st]:starts[st] + dt, starts[sf]:starts[sf] + df] = \
                a["op_data"][o:o + df * dt].reshape(dt, df, order="F")
        names = {0: lambda y, s: ("c", y, s), 1: lambda y, s: ("sz", y), 2: lambda y, s: ("sp", y)}
        assert len(keys) == len(B.edge)
        for k in keys:
            name = names[k[0]](k[1], k[2])
            assert np.array_equal(ops[k], _edge_matrix_from_bits(B, name)), (case, B.side, name)
        # the Hamiltonian blocks are the block's own, sector by sector
        H = sp.csr_matrix(B.H).toarray()
        off = 0
        for i, d in enumerate(dims):
            d = int(d)
            blk = a["H"][off:off + d * d].reshape(d, d, order="F")
            assert np.array_equal(blk, H[starts[i]:starts[i] + d, starts[i]:starts[i] + d])
            off += d * d


def _lattice_in_packed_order(sb, model, length, Q):
    occ = sb.occupation_of_packed()
    H, basis = lattice_hamiltonian(model, length, Q)
    pos = np.searchsorted(basis, occ)
    assert np.array_equal(basis[pos], occ)
    return H[pos][:, pos]


@pytest.mark.parametrize("model,k,Q,length", [
    (Model("hubbard", 2, t=1.0, U=4.0), 1, (4, 4), 4),
    (Model("hubbard", 2, t=1.0, U=4.0), 1, (3, 4), 4),
    (Model("hubbard", 3, t=1.0, U=2.0), 1, (2, 3), 4),
    (Model("heisenberg", 2, J=1.0), 2, (6, 0), 6),
])
def test_exact_blocks_through_the_file_equal_lattice(tmp_path, monkeypatch, model, k, Q, length):
    """Exact blocks written to and read from a block file build the
    superblock of Eq. (1) that equals the brute-force lattice Hamiltonian
    element by element (fermion strings of the stored operators included)."""
    L, R = exact_block(model, k, "L"), exact_block(model, k, "R")
    L2, R2, _ = _roundtrip(tmp_path, monkeypatch, L, R)
    L2.occ, R2.occ = L.occ, R.occ           # the file holds no occupation bits
    sb = Superblock(L2, R2, Q)
    Hlat = _lattice_in_packed_order(sb, model, length, Q)
    assert abs(sb.explicit() - Hlat).max() < 1e-13


@pytest.mark.slow
def test_exact_two_column_hubbard_blocks_through_the_file_lattice_energy(tmp_path, monkeypatch):
    """2x6 Hubbard at half filling from exact two-column blocks (256 states)
    read back from a block file: the superblock's ground energy equals the
    lattice's (853,776 states, ARPACK on both)."""
    from scipy.sparse.linalg import eigsh
    model = Model("hubbard", 2, t=1.0, U=5.0)
    L, R = exact_block(model, 2, "L"), exact_block(model, 2, "R")
    L2, R2, _ = _roundtrip(tmp_path, monkeypatch, L, R)
    sb = Superblock(L2, R2, (6, 6))
    Hlat, _ = lattice_hamiltonian(model, 6, (6, 6))
    assert Hlat.shape[0] == sb.N == 853776
    v0 = np.random.default_rng(3).standard_normal(sb.N)
    from scipy.sparse.linalg import LinearOperator
    e_sb = eigsh(LinearOperator((sb.N, sb.N), matvec=sb.hv_factored, dtype=np.float64), k=1, which="SA",
                 v0=v0, tol=1e-12)[0][0]
    e_lat = eigsh(Hlat, k=1, which="SA", v0=v0, tol=1e-12)[0][0]
    assert abs(e_sb - e_lat) <= 1e-10 * abs(e_lat)


# ---------------------------------------------------------------------- the bound
@pytest.mark.parametrize("model,k,Q,length", [
    (Model("heisenberg", 2, J=1.0), 2, (6, 0), 6),
    (Model("hubbard", 2, t=1.0, U=8.0), 1, (4, 4), 4),
    (Model("hubbard", 3, t=1.0, U=2.0), 1, (2, 3), 4),
])
def test_abs_bound_mode_f_equals_mode_x_and_bounds(model, k, Q, length):
    sb = Superblock(exact_block(model, k, "L"), exact_block(model, k, "R"), Q)
    v = np.random.default_rng(4).standard_normal(sb.N)
    b = sb.hv_abs_bound(v)
    bx = sb.explicit(absolute=True) @ np.abs(v)
    assert np.abs(b - bx).max() <= 1e-13 * max(1.0, np.abs(bx).max())
    # triangle inequality: |H v| <= |H_lattice| |v| <= bound, element by element
    Hlat = _lattice_in_packed_order(sb, model, length, Q)
    a = abs(Hlat) @ np.abs(v)
    assert np.all(np.abs(sb.hv_factored(v)) <= a + 1e-12)
    assert np.all(a <= b + 1e-12)


@pytest.mark.parametrize("case,Q", [("hubbard_truncated", (6, 6)), ("heisenberg_truncated", (6, 0))])
def test_abs_bound_truncated_blocks_mode_x(case, Q):
    L, R = BLOCK_CASES[case]()
    sb = Superblock(L, R, Q)
    v = np.random.default_rng(5).standard_normal(sb.N)
    b = sb.hv_abs_bound(v)
    bx = sb.explicit(absolute=True) @ np.abs(v)
    assert np.abs(b - bx).max() <= 1e-12 * np.abs(bx).max()
    assert np.all(np.abs(sb.hv_factored(v)) <= b * (1 + 1e-12) + 1e-300)


# ---------------------------------------------------------------------- the checker
@pytest.mark.slow
def test_checker_catches_one_bad_tile_the_norm_misses():
    """4-leg Heisenberg m=1000 (N = 4.2e7): a 1% error on one 16 x 16 tile of
    the smallest sector block with both sides >= 16 fails the element-wise
    bar (and its sector's norm); so does 1% on the whole smallest sector
    block, which the global relative 2-norm bar of 1e-5 misses; an
    FP32-sized perturbation of every element passes."""
    from helpers import oracle_superblock, rel_err
    osb = oracle_superblock(W.HEISENBERG_4X16_M1000)
    v = W.random_vector(osb.N, 1000)
    ref = osb.hv_factored(v)
    bound = osb.hv_abs_bound(v)
    secs = osb.sector_table()
    rng = np.random.default_rng(6)
    ok = ref + bound * 1e-7 * rng.uniform(-1, 1, size=ref.size)
    rep = parity(ok, ref, bound, 1e-5, secs)
    assert rep["n_bad"] == 0 and rep["worst_sector"] <= 1e-5
    q, dL, dR, o = min((s for s in secs if s[1] >= 16 and s[2] >= 16), key=lambda s: s[1] * s[2])
    bad = ref.copy()
    blk = bad[o:o + dL * dR].reshape(dR, dL)          # column-major d_L x d_R block, transposed view
    blk[:16, :16] *= 1.01
    rep = parity(bad, ref, bound, 1e-5, secs)
    print(f"sector {q} ({dL}x{dR}): global rel norm of the planted error {rel_err(bad, ref):.2e}, "
          f"elements over {rep['n_bad']}, worst sector {rep['worst_sector']:.2e}")
    assert rep["n_bad"] > 0
    assert rep["worst_sector"] > 1e-5
    # 1% on the whole of the smallest sector block: below the global 2-norm bar
    q, dL, dR, o = min(secs, key=lambda s: s[1] * s[2])
    bad = ref.copy()
    bad[o:o + dL * dR] *= 1.01
    rep = parity(bad, ref, bound, 1e-5, secs)
    print(f"sector {q} ({dL}x{dR}): global rel norm {rel_err(bad, ref):.2e}, elements over {rep['n_bad']}")
    assert rel_err(bad, ref) < 1e-5
    assert rep["n_bad"] > 0 and rep["worst_sector"] > 1e-5


# ---------------------------------------------------------------------- golden energies
def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _in_use():
    names = [wl for wl in W.WORKLOADS.values()] + list(W.batch64())
    g = _golden()
    return [(wl, g[wl.name]) for wl in names if wl.name in g]


def test_golden_records_cover_the_workloads_in_use():
    g = _golden()
    for wl in list(W.WORKLOADS.values()) + list(W.batch64()):
        assert wl.name in g, wl.name
        assert g[wl.name]["block_hash"] == W.block_file_hash(wl.name), wl.name


def test_golden_residuals_are_small():
    for wl, rec in _in_use():
        assert rec["residual"] <= 1e-12 * abs(rec["E0"]), wl.name


def test_golden_lattice_ed_where_recorded():
    g = _golden()
    rec = g[W.HEISENBERG_2X6_M16.name]
    assert rec["E0_lattice_ed"] is not None
    assert abs(rec["E0"] - rec["E0_lattice_ed"]) <= 1e-12 * abs(rec["E0_lattice_ed"])
    for name, rec in g.items():
        if rec.get("E0_lattice_ed") is not None:
            assert abs(rec["E0"] - rec["E0_lattice_ed"]) <= 1e-12 * abs(rec["E0_lattice_ed"]), name


def _with_second_figure():
    """The single-superblock workloads, and the batch problems on the drawn
    12-column lattice whose references exist (their record is written with
    both figures)."""
    g = _golden()
    wls = list(W.WORKLOADS.values()) + list(W.batch64(W.BATCH_LENGTH_DRAWN))
    return [(wl, g[wl.name]) for wl in wls if wl.name in g]


def test_golden_second_figure():
    """Every reference has a second figure: the oracle's own Lanczos (small
    targets) or a Kato-Temple bracket from a second ARPACK run (large ones)."""
    for wl, rec in _with_second_figure():
        if "E0_lanczos" in rec:
            assert abs(rec["E0"] - rec["E0_lanczos"]) <= 1e-12 * abs(rec["E0"]), wl.name
            continue
        lo = rec.get("E0_kato_temple_lower")
        assert lo is not None, f"{wl.name}: no second figure"
        assert lo <= rec["E0"] + 1e-12 * abs(rec["E0"]), wl.name
        assert rec["E0"] - lo <= 1e-12 * abs(rec["E0"]), wl.name
        if "E0_second" in rec:
            assert abs(rec["E0_second"] - rec["E0"]) <= 1e-12 * abs(rec["E0"]), wl.name
