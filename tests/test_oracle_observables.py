"""Pins of the local observables of Eqs. (2)-(4) (oracle.observables, CPU).

* With exact blocks the superblock ground state is the lattice ground state,
  so the densities the superblock state gives on its two explicit columns
  equal the brute-force lattice state's on those lattice columns.
* The lattice densities sum to the particle numbers of the sector.
* Lieb-Mattis: the half-filled Hubbard ladder and the Heisenberg ladder have a
  singlet ground state, so s(x, y) = 0 on every site (Eq. (3)); the hole
  density of a half-filled ladder averages to 0.
"""
import numpy as np
import pytest

from oracle.blocks import exact_block
from oracle.lattice import lattice_hamiltonian
from oracle.local import Model
from oracle.observables import (column_densities, hole_and_spin_density, lattice_densities,
                                staggered_max)
from oracle.superblock import Superblock

CASES = [
    (Model("hubbard", 2, t=1.0, U=4.0), 1, (4, 4), 4),
    (Model("hubbard", 2, t=1.0, U=8.0), 1, (3, 4), 4),        # one hole, S_z = -1/2
    (Model("hubbard", 1, t=1.0, U=3.0), 2, (2, 3), 6),
    (Model("heisenberg", 2, J=1.0), 2, (6, 0), 6),
    (Model("heisenberg", 3, J=1.0), 1, (7, 0), 4),            # S_z = 1
]


def _ground(H):
    from scipy.sparse.linalg import eigsh
    if H.shape[0] <= 1000:
        w, v = np.linalg.eigh(H.toarray())
    else:
        w, v = eigsh(H, k=2, which="SA", tol=1e-14, v0=np.ones(H.shape[0]))
        o = np.argsort(w)
        w, v = w[o], v[:, o]
    assert w[1] - w[0] > 1e-8, "degenerate ground state"
    return v[:, 0]


@pytest.mark.parametrize("model,k,Q,length", CASES)
def test_column_densities_equal_lattice(model, k, Q, length):
    sb = Superblock(exact_block(model, k, "L"), exact_block(model, k, "R"), Q)
    psi = _ground(sb.explicit())
    n_sb = column_densities(sb, psi)
    H, basis = lattice_hamiltonian(model, length, Q)
    n_lat = lattice_densities(model, length, basis, _ground(H))
    x2 = sb.L.ncols
    assert np.abs(n_sb[0] - n_lat[x2]).max() < 1e-10
    assert np.abs(n_sb[1] - n_lat[x2 + 1]).max() < 1e-10
    # particle numbers (spin model: up spins and down spins)
    tot = n_lat.sum(axis=(0, 1))
    nsites = model.legs * length
    want = (Q[0], Q[1]) if model.fermionic else (Q[0], nsites - Q[0])
    assert np.allclose(tot, want, atol=1e-10)


@pytest.mark.parametrize("model,k,Q,length", [CASES[0], CASES[3],
                                               (Model("hubbard", 1, t=1.0, U=3.0), 2, (3, 3), 6)])
def test_lieb_mattis_zero_spin_density(model, k, Q, length):
    sb = Superblock(exact_block(model, k, "L"), exact_block(model, k, "R"), Q)
    psi = _ground(sb.explicit())
    h, s = hole_and_spin_density(column_densities(sb, psi))
    assert np.abs(s).max() < 1e-10
    assert staggered_max(s).max() < 1e-10
    if model.fermionic and Q[0] + Q[1] == model.legs * length:
        assert abs(h.mean()) < 1e-10


def test_spin_density_of_a_polarised_sector_is_not_zero():
    """A planted mistake the Lieb-Mattis check must not hide: in the S_z = 1
    sector the spin density is nonzero and sums to twice the magnetisation."""
    model, k, Q, length = CASES[4]
    sb = Superblock(exact_block(model, k, "L"), exact_block(model, k, "R"), Q)
    H, basis = lattice_hamiltonian(model, length, Q)
    n_lat = lattice_densities(model, length, basis, _ground(H))
    _, s = hole_and_spin_density(n_lat)
    assert abs(s.sum() - (2 * Q[0] - model.legs * length)) < 1e-10
    assert staggered_max(s).max() > 1e-3
