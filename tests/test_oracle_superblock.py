"""Pins of the Eq. (1) superblock construction and its products (oracle.superblock).

* With exact blocks the superblock Hamiltonian must equal the brute-force
  lattice Hamiltonian element by element, under the basis map
  |i1 i2 i3 i4> -> lattice occupation bits (the block states are products of
  creators in global mode order, so no extra sign appears).
* With truncated blocks it must equal the exact one projected by the
  truncation isometries.
* The paper's index maps are checked against plain reshapes, and the two
  products (explicit sparse H, and H_l V + V H_r^T + H_c V_c) against each other.
* Planted mistakes (in the oracle, on the CPU) must be caught.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle.blocks as ob
import oracle.local as ol
import oracle.superblock as osb
from oracle.blocks import exact_block, left_half, right_half, block_from_half, truncate_half
from oracle.dmrg import reduced_density_matrices
from oracle.lattice import lattice_hamiltonian, ground_energy
from oracle.local import Model, make_column
from oracle.superblock import Superblock

CASES = [
    (Model("heisenberg", 2, J=1.0), 2, (6, 0), 6),          # the 2x6 ladder's geometry
    (Model("heisenberg", 2, J=1.0), 2, (7, 0), 6),
    (Model("heisenberg", 3, J=0.7), 1, (6, 0), 4),
    (Model("hubbard", 2, t=1.0, U=8.0), 1, (4, 4), 4),
    (Model("hubbard", 2, t=1.0, U=4.0), 1, (3, 4), 4),
    (Model("hubbard", 1, t=1.0, U=3.0), 2, (3, 2), 6),
    (Model("hubbard", 3, t=1.0, U=2.0), 1, (2, 3), 4),
]


def lattice_in_packed_order(sb, model, length, Q):
    occ = sb.occupation_of_packed()
    H, basis = lattice_hamiltonian(model, length, Q)
    pos = np.searchsorted(basis, occ)
    assert np.array_equal(basis[pos], occ), "superblock basis is not the lattice sector"
    assert pos.size == basis.size
    return H[pos][:, pos]


@pytest.mark.parametrize("model,k,Q,length", CASES)
def test_eq1_equals_lattice_elementwise(model, k, Q, length):
    sb = Superblock(exact_block(model, k, "L"), exact_block(model, k, "R"), Q)
    Hx = sb.explicit()
    Hlat = lattice_in_packed_order(sb, model, length, Q)
    assert abs(Hx - Hlat).max() < 1e-13
    v = np.random.default_rng(1).standard_normal(sb.N)
    assert np.abs(sb.hv_factored(v) - Hlat @ v).max() < 1e-12


def test_index_maps_against_reshape():
    rng = np.random.default_rng(0)
    m, n = 5, 3
    v = rng.standard_normal((m * n) ** 2)
    V = v.reshape(m * n, m * n, order="F")
    T = v.reshape(m, n, m, n, order="F")           # axes (i1, i2, i4, i3)
    Vc = np.transpose(T, (1, 3, 0, 2)).reshape(n * n, m * m, order="F")
    for _ in range(200):
        i1, i4 = rng.integers(1, m + 1, size=2)
        i2, i3 = rng.integers(1, n + 1, size=2)
        idx = (i3 - 1) * m * m * n + (i4 - 1) * m * n + (i2 - 1) * m + i1      # 1-based
        assert V[(i2 - 1) * m + i1 - 1, (i3 - 1) * m + i4 - 1] == v[idx - 1]
        assert Vc[(i3 - 1) * n + i2 - 1, (i4 - 1) * m + i1 - 1] == v[idx - 1]
    # the V_c map of the oracle is a bijection and agrees with the reshape above
    sb = Superblock(exact_block(Model("heisenberg", 2), 1, "L"), exact_block(Model("heisenberg", 2), 1, "R"), (4, 0))
    vc = sb.vc_index_of_full()
    assert np.array_equal(np.sort(vc), np.arange(vc.size))
    x = rng.standard_normal(vc.size)
    Xc = np.zeros_like(x); Xc[vc] = x
    T = x.reshape(4, 4, 4, 4, order="F")
    assert np.array_equal(Xc, np.transpose(T, (1, 3, 0, 2)).reshape(-1, order="F"))


def test_central_forms_agree():
    """H_c V_c (paper) equals sum_k a_k V b_k^T written out on the full space."""
    model = Model("hubbard", 2, t=1.0, U=2.0)
    col = make_column(model)
    L, R = exact_block(model, 1, "L"), exact_block(model, 1, "R")
    sb = Superblock(L, R, (3, 3))
    m, n = sb.m, sb.n
    v = np.random.default_rng(2).standard_normal(sb.N)
    vf = sb.unpack(v)
    V = vf.reshape(m * n, m * n, order="F")
    Im = np.eye(m)
    W = np.zeros_like(V)
    for coef, A, B in ol.bond_terms(model, col.ops, col.parity, col.ops):
        W += coef * np.kron(A.toarray(), Im) @ V @ np.kron(B.toarray(), Im).T
    # H_c part only: subtract the H_l, H_r parts of mode F
    w_all = sb.hv_factored(v)
    w_lr = np.zeros_like(v)
    for (q, r, c, o), (hl, hr) in zip(sb.sectors, sb.dense_sectors()):
        Vs = v[o:o + r.size * c.size].reshape(c.size, r.size).T
        w_lr[o:o + r.size * c.size] = (hl @ Vs + Vs @ hr.T).T.reshape(-1)
    assert np.abs(sb.pack(W.reshape(-1, order="F")) - (w_all - w_lr)).max() < 1e-13


def _project_full(sbx, UL, UR):
    n = sbx.n
    In = sp.identity(n, format="csr")
    return sp.kron(sp.kron(In, UR), sp.kron(In, UL)).tocsr()


@pytest.mark.parametrize("model,k,mk,Q", [
    (Model("heisenberg", 2, J=1.0), 2, 10, (8, 0)),
    (Model("hubbard", 1, t=1.0, U=4.0), 3, 20, (4, 4)),
])
def test_truncated_blocks_are_projections(model, k, mk, Q):
    col = make_column(model)
    Lk, Rk = exact_block(model, k, "L"), exact_block(model, k, "R")
    # a state to define the density matrices: the ground state one size down
    sb0 = Superblock(exact_block(model, k - 1, "L"), exact_block(model, k - 1, "R"),
                     (Q[0] - model.legs, Q[1] - (model.legs if model.fermionic else 0)))
    psi = np.linalg.eigh(sb0.explicit().toarray())[1][:, 0]
    rhoL, rhoR, rows_of, cols_of = reduced_density_matrices(sb0, psi)
    Lt, _, _, specL, UL = truncate_half(sb0.left, rhoL, rows_of, mk)
    Rt, _, _, specR, UR = truncate_half(sb0.right, rhoR, cols_of, mk)
    assert Lt.dim == mk and Rt.dim == mk
    # the exact blocks are sorted versions of the same halves
    ordL = np.lexsort((np.arange(sb0.left.dim), sb0.left.qn[:, 1], sb0.left.qn[:, 0]))
    ordR = np.lexsort((np.arange(sb0.right.dim), sb0.right.qn[:, 1], sb0.right.qn[:, 0]))
    UL, UR = UL.tocsr()[ordL], UR.tocsr()[ordR]
    Hex = Superblock(Lk, Rk, Q).explicit(full_space=True)
    Htr = Superblock(Lt, Rt, Q).explicit(full_space=True)
    P = _project_full(Superblock(Lk, Rk, Q), UL, UR)
    assert abs(Htr - (P.T @ Hex @ P)).max() < 1e-12
    # Schmidt: rho_L and rho_R share their nonzero spectrum
    a = np.sort(specL)[::-1][:20]; b = np.sort(specR)[::-1][:20]
    assert np.allclose(a, b, atol=1e-12)


def test_density_matrix_invariants():
    model = Model("hubbard", 2, t=1.0, U=4.0)
    sb = Superblock(exact_block(model, 1, "L"), exact_block(model, 1, "R"), (4, 4))
    psi = np.random.default_rng(5).standard_normal(sb.N); psi /= np.linalg.norm(psi)
    rhoL, rhoR, _, _ = reduced_density_matrices(sb, psi)
    trL = sum(np.trace(r) for r in rhoL.values()); trR = sum(np.trace(r) for r in rhoR.values())
    assert abs(trL - 1) < 1e-12 and abs(trR - 1) < 1e-12
    eL = np.sort(np.concatenate([np.linalg.eigvalsh(r) for r in rhoL.values()]))
    eR = np.sort(np.concatenate([np.linalg.eigvalsh(r) for r in rhoR.values()]))
    assert eL.min() > -1e-14 and eR.min() > -1e-14
    nz = min(eL.size, eR.size)
    assert np.allclose(eL[-nz:], eR[-nz:], atol=1e-13)


def test_dmrg_without_truncation_is_exact():
    from oracle.dmrg import infinite_system
    model = Model("heisenberg", 2, J=1.0)
    L, R, hist = infinite_system(model, 2, 10 ** 6, lambda ns: (ns // 2, 0))
    sb = Superblock(L, R, (6, 0))
    e_sb = np.linalg.eigvalsh(sb.explicit().toarray())[0]
    e_lat = ground_energy(lattice_hamiltonian(model, 6, (6, 0))[0])[0]
    assert abs(e_sb - e_lat) < 1e-12


@pytest.mark.parametrize("model,length,m,Q", [
    (Model("hubbard", 1, t=1.0, U=4.0), 10, 16, (5, 5)),
    (Model("heisenberg", 2, J=1.0), 8, 12, (8, 0)),
])
def test_truncated_dmrg_is_variational(model, length, m, Q):
    from oracle.dmrg import infinite_system, solve
    bc = (length - 2) // 2
    tgt = (lambda ns: (ns // 2, ns // 2)) if model.fermionic else (lambda ns: (ns // 2, 0))
    L, R, hist = infinite_system(model, bc, m, tgt)
    assert L.dim == m
    sb = Superblock(L, R, Q)
    E, _, _ = solve(sb, tol=1e-14)
    Eex = ground_energy(lattice_hamiltonian(model, length, Q)[0])[0]
    assert E >= Eex - 1e-10
    assert E - Eex < 5e-2 * abs(Eex)


# ------------------------------------------------------------ planted mistakes
def _eq1_mismatch(model, k, Q, length):
    sb = Superblock(exact_block(model, k, "L"), exact_block(model, k, "R"), Q)
    Hx = sb.explicit()
    Hlat = lattice_in_packed_order(sb, model, length, Q)
    return abs(Hx - Hlat).max()


def test_mutation_dropped_string_is_caught(monkeypatch):
    orig = ol.bond_terms

    def no_string(model, ops_x, parity_x, ops_y):
        return orig(model, ops_x, np.ones_like(parity_x), ops_y)

    monkeypatch.setattr(ob, "bond_terms", no_string)
    monkeypatch.setattr(osb, "bond_terms", no_string)
    assert _eq1_mismatch(Model("hubbard", 2, t=1.0, U=4.0), 1, (3, 4), 4) > 0.5


def test_mutation_central_kron_order_is_caught(monkeypatch):
    real = sp.kron

    class Swapped(Superblock):
        def __init__(self, *a, **kw):
            super().__init__(*a, **kw)
            n = self.n
            Hc = sp.csr_matrix((n * n, n * n))
            for coef, A, B in ol.bond_terms(self.model, self.col.ops, self.col.parity, self.col.ops):
                Hc = Hc + coef * real(A, B)          # wrong: i2 slow instead of i3 slow
            self.H_c = sp.csr_matrix(Hc)

    # (the spin model's bond is symmetric under the swap; the fermion string is not)
    model = Model("hubbard", 2, t=1.0, U=4.0)
    sb = Swapped(exact_block(model, 1, "L"), exact_block(model, 1, "R"), (3, 4))
    Hlat = lattice_in_packed_order(sb, model, 4, (3, 4))
    assert abs(sb.explicit() - Hlat).max() > 0.1


def test_mutation_transposed_vector_map_is_caught():
    model = Model("heisenberg", 2, J=1.0)
    sb = Superblock(exact_block(model, 2, "L"), exact_block(model, 2, "R"), (6, 0))
    v = np.random.default_rng(0).standard_normal(sb.N)
    good = sb.hv_factored(v)
    # V stored row-major instead of column-major in every sector
    w = np.zeros_like(v)
    for (q, r, c, o), (hl, hr) in zip(sb.sectors, sb.dense_sectors()):
        V = v[o:o + r.size * c.size].reshape(r.size, c.size)
        w[o:o + r.size * c.size] = (hl @ V + V @ hr.T).reshape(-1)
    assert np.abs(w - good).max() > 0.1


def test_mutation_wrong_hopping_sign_in_column_is_caught(monkeypatch):
    orig = ol.hubbard_column

    def bad(legs, t, U):
        col = orig(legs, t, U)
        a, c = col.ops[("c", 0, 0)], col.ops[("c", 1, 0)]
        col.H = sp.csr_matrix(col.H + 2 * t * (a.T @ c + c.T @ a))   # rung hopping sign flipped for up spins only
        return col

    monkeypatch.setattr(ol, "hubbard_column", bad)
    assert _eq1_mismatch(Model("hubbard", 2, t=1.0, U=4.0), 1, (3, 4), 4) > 0.5


@pytest.mark.parametrize("model,k,Q,length", CASES[:1] + CASES[3:5] + CASES[6:])
def test_column_offdiagonal_part_as_gathers(model, k, Q, length):
    """The halves without the explicit columns' off-diagonal terms, plus those
    terms applied as scaled copies of V's rectangles (row runs of one
    column-2 state moved to another, column runs of one column-3 state
    likewise, the weights read from the column Hamiltonian itself), give
    H_l V + V H_r^T; the removed part of each sector is exactly the column
    Hamiltonian's off-diagonal entries between states with equal block
    states, and it conserves the sectors."""
    L, R = exact_block(model, k, "L"), exact_block(model, k, "R")
    sb = Superblock(L, R, Q)
    m, n = sb.m, sb.n
    hcol = sb.col.H.toarray()
    v = np.random.default_rng(4).standard_normal(sb.N)
    w_lr, w_split = np.zeros(sb.N), np.zeros(sb.N)
    for (q, r, c, o), (hl, hr), (hl0, hr0) in zip(sb.sectors, sb.dense_sectors(),
                                                 sb.dense_sectors(column_offdiagonal=False)):
        Vs = v[o:o + r.size * c.size].reshape(c.size, r.size).T
        w_lr[o:o + r.size * c.size] = (hl @ Vs + Vs @ hr.T).T.reshape(-1)
        W = hl0 @ Vs + Vs @ hr0.T
        # the removed part, element by element from the column Hamiltonian
        for idx, H, H0 in ((r, hl, hl0), (c, hr, hr0)):
            a, b = idx // m, idx % m
            want = np.where((b[:, None] == b[None, :]) & (a[:, None] != a[None, :]), hcol[a[:, None], a[None, :]], 0.0)
            assert np.array_equal(H - H0, want)
        # the same part as gathers over rows (column 2) and columns (column 3)
        a_r, b_r = r // m, r % m
        a_c, b_c = c // m, c % m
        for i in range(r.size):
            for j in range(r.size):
                if b_r[i] == b_r[j] and a_r[i] != a_r[j] and hcol[a_r[i], a_r[j]] != 0:
                    W[i, :] += hcol[a_r[i], a_r[j]] * Vs[j, :]
        for i in range(c.size):
            for j in range(c.size):
                if b_c[i] == b_c[j] and a_c[i] != a_c[j] and hcol[a_c[i], a_c[j]] != 0:
                    W[:, i] += hcol[a_c[i], a_c[j]] * Vs[:, j]
        w_split[o:o + r.size * c.size] = W.T.reshape(-1)
    assert np.abs(w_split - w_lr).max() <= 1e-13 * max(1.0, np.abs(w_lr).max())
