"""Pins of the finite-system sweeps and the wavefunction transformation
(oracle.sweeps, CPU; the sweeps of Fig. 3's energy-versus-sweep study).

* The transformation against a brute-force loop over every index of a small
  state (the einsum / reshape bookkeeping).
* Its exact identities: the start vector's squared norm is the weight the
  new block keeps (1 - the truncation error of the step before), and the
  start vector's energy is never below the superblock's ground energy
  (variational in the superblock's space).
* Every sweep energy lies above the lattice ground energy (the DMRG energy is
  variational) and with m = 64 on the 2 x 10 Heisenberg ladder the sweeps
  reach the lattice ground energy.
* The transformed state starts the solver closer to the ground state than a
  random vector: fewer Lanczos products to the same bar.
"""
import numpy as np
import pytest

from oracle.lattice import ground_energy, lattice_hamiltonian
from oracle.local import Model
from oracle.superblock import Superblock
from oracle.sweeps import _grow, _solve, finite_sweeps, infinite_blocks, sweep_positions, wavefunction_transform

HEIS2 = Model("heisenberg", 2, J=1.0)
HUB2 = Model("hubbard", 2, t=1.0, U=4.0)


def sz0(ns):
    return (ns // 2, 0)


def half(ns):
    return (ns // 2, ns // 2)


def lattice_e0(model, L, qn):
    r = lattice_hamiltonian(model, L, qn)
    H = r[0] if isinstance(r, tuple) else r
    return float(np.asarray(ground_energy(H)).reshape(-1)[0])


def test_sweep_positions():
    st = sweep_positions(10, 2, 2)
    assert st[0] == (4, 0) and st[-1] == (4, -1)
    pos = [p for p, _ in st]
    assert min(pos) == 2 and max(pos) == 6
    # each move goes one column in its direction
    for (p, d), (q, _) in zip(st[:-1], st[1:]):
        assert q == p + (1 if d == 0 else -1)
    assert len(st) == 2 * 2 * (6 - 2) + 1


@pytest.mark.parametrize("direction", [0, 1])
def test_transform_against_index_loops(direction):
    """2 x 8 Heisenberg, m = 16: one step of each direction recomputed by
    plain loops over (i1, i2, i3, i4) and the new indices."""
    L, m = 8, 16
    left, right, sb, E, psi, _ = infinite_blocks(HEIS2, 3, m, sz0)
    target = sz0(2 * L)
    l = 3
    if direction == 0:
        newL, _ = _grow(sb, psi, m, "L")
        nxt = Superblock(newL, right[L - l - 3], target)
        Un, Uo = newL.U, right[L - l - 2].U
    else:
        newR, _ = _grow(sb, psi, m, "R")
        nxt = Superblock(left[l - 1], newR, target)
        Un, Uo = newR.U, left[l].U
    got = wavefunction_transform(sb, psi, nxt, Un, Uo, direction)
    n, ma, mb = sb.n, sb.m, nxt.m
    V = sb.unpack(psi).reshape(n * ma, n * ma, order="F")
    W = np.zeros((n * mb, n * mb))
    nz = np.argwhere(np.abs(V) > 0)
    for r, c in nz:
        i2, i1 = divmod(r, ma)
        i3, i4 = divmod(c, ma)
        x = V[r, c]
        if direction == 0:
            # psi'[(i3, j1), (j3, j4)] += Un[(i2, i1), j1] psi Uo[(j3, j4), i4]
            for j1 in np.flatnonzero(Un[r]):
                for q in np.flatnonzero(Uo[:, i4]):
                    W[i3 * mb + j1, q] += Un[r, j1] * x * Uo[q, i4]
        else:
            # psi'[(j2, j1), (i2, j4)] += Uo[(j2, j1), i1] psi Un[(i3, i4), j4]
            for j4 in np.flatnonzero(Un[c]):
                for q in np.flatnonzero(Uo[:, i1]):
                    W[q, i2 * mb + j4] += Uo[q, i1] * x * Un[c, j4]
    want = nxt.pack(W.reshape(-1, order="F"))
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.fixture(scope="module")
def heis_2x10_m16():
    return finite_sweeps(HEIS2, 10, 16, sz0, l_min=2, nsweeps=2)


def test_start_vector_norm_is_the_kept_weight(heis_2x10_m16):
    for prev, rec in zip(heis_2x10_m16[:-1], heis_2x10_m16[1:]):
        assert abs(rec["guess_norm"] ** 2 - (1.0 - prev["trunc"])) <= 1e-12


def test_start_vector_energy_is_variational(heis_2x10_m16):
    for rec in heis_2x10_m16:
        assert rec["guess_energy"] >= rec["energy"] - 1e-12 * abs(rec["energy"])


def test_sweep_energies_above_the_lattice_ground_energy(heis_2x10_m16):
    e0 = lattice_e0(HEIS2, 10, (10, 0))
    for rec in heis_2x10_m16:
        assert rec["energy"] >= e0 - 1e-10 * abs(e0)
    # the sweeps converge: the middle position's energy changes by little in the last sweep
    mid = [r["energy"] for r in heis_2x10_m16 if r["position"] == 4]
    assert abs(mid[-1] - mid[-2]) <= 1e-8 * abs(e0)


def test_sweeps_reach_the_lattice_ground_energy_with_enough_states():
    recs = finite_sweeps(HEIS2, 10, 64, sz0, l_min=3, nsweeps=1)
    e0 = lattice_e0(HEIS2, 10, (10, 0))
    for rec in recs:
        assert rec["energy"] >= e0 - 1e-10 * abs(e0)
    assert abs(recs[-1]["energy"] - e0) <= 1e-8 * abs(e0)


def test_hubbard_sweeps_variational():
    recs = finite_sweeps(HUB2, 6, 16, half, l_min=1, nsweeps=2)
    e0 = lattice_e0(HUB2, 6, (6, 6))
    for prev, rec in zip(recs[:-1], recs[1:]):
        assert abs(rec["guess_norm"] ** 2 - (1.0 - prev["trunc"])) <= 1e-12
    for rec in recs:
        assert rec["energy"] >= e0 - 1e-10 * abs(e0)
        assert rec["guess_energy"] >= rec["energy"] - 1e-12 * abs(rec["energy"])


def test_transformed_start_needs_fewer_products(heis_2x10_m16):
    """At every step after the first, the transformed state reaches the bar in
    fewer products than a random start on the same superblock would."""
    left, right, sb, _, _, _ = infinite_blocks(HEIS2, 4, 16, sz0)
    _, _, info = _solve(sb, np.random.default_rng(5).standard_normal(sb.N), 1e-13)   # the sweeps' own bar
    random_products = info["iterations"]
    assert max(r["products"] for r in heis_2x10_m16[1:]) < random_products
