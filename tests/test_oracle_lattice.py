"""Pins of the brute-force lattice Hamiltonians (oracle.lattice).

Closed forms and symmetries fixed by the mathematics, not by the oracle:
a dropped hopping sign, a wrong Jordan-Wigner string, a missing U term or a
wrong spin-flip amplitude each fail at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.lattice import bonds, ground_energy, hubbard_hamiltonian, heisenberg_hamiltonian
from oracle.lanczos import lanczos_ground


def free_fermion_energy(legs, length, t, nup, ndn):
    """U=0: fill the OBC tight-binding levels -2t[cos(pi a/(s+1)) + cos(pi b/(L+1))]."""
    eps = sorted(-2 * t * (math.cos(math.pi * a / (legs + 1)) + math.cos(math.pi * b / (length + 1)))
                 for a in range(1, legs + 1) for b in range(1, length + 1))
    return sum(eps[:nup]) + sum(eps[:ndn])


@pytest.mark.parametrize("U", [0.0, 1.0, 4.0, 8.0, 10.0])
@pytest.mark.parametrize("geom", [(1, 2), (2, 1)])
def test_two_site_hubbard_closed_form(U, geom):
    H, _ = hubbard_hamiltonian(geom[0], geom[1], 1.0, U, 1, 1)
    E = np.linalg.eigvalsh(H.toarray())[0]
    assert abs(E - (U - math.sqrt(U * U + 16.0)) / 2) < 1e-12


@pytest.mark.parametrize("legs,length,nup,ndn", [(2, 3, 3, 2), (2, 4, 4, 4), (3, 2, 3, 3),
                                                  (2, 4, 3, 1), (1, 6, 3, 3), (3, 3, 4, 5)])
def test_free_fermions(legs, length, nup, ndn):
    H, _ = hubbard_hamiltonian(legs, length, 1.0, 0.0, nup, ndn)
    E = ground_energy(H)[0]
    assert abs(E - free_fermion_energy(legs, length, 1.0, nup, ndn)) < 1e-10


def test_free_fermion_full_spectrum_single_particle():
    # one particle: the whole spectrum is the tight-binding band
    H, _ = hubbard_hamiltonian(2, 5, 1.0, 3.0, 1, 0)
    ev = np.linalg.eigvalsh(H.toarray())
    ref = sorted(-2 * (math.cos(math.pi * a / 3) + math.cos(math.pi * b / 6))
                 for a in (1, 2) for b in range(1, 6))
    assert np.allclose(ev, ref, atol=1e-12)


@pytest.mark.parametrize("nup,ndn", [(2, 2), (3, 3), (4, 3), (2, 5)])
def test_atomic_limit(nup, ndn):
    U = 5.0
    H, _ = hubbard_hamiltonian(2, 3, 0.0, U, nup, ndn)
    E = np.linalg.eigvalsh(H.toarray())[0]
    assert abs(E - U * max(0, nup + ndn - 6)) < 1e-12


def test_heisenberg_closed_forms():
    H, _ = heisenberg_hamiltonian(1, 2, 1.0, 1)
    assert abs(np.linalg.eigvalsh(H.toarray())[0] + 0.75) < 1e-14
    H, _ = heisenberg_hamiltonian(2, 2, 1.0, 2)           # 2x2 = 4-site ring
    assert abs(np.linalg.eigvalsh(H.toarray())[0] + 2.0) < 1e-13
    for legs, length in [(2, 6), (4, 2), (3, 3)]:
        ns = legs * length
        H, _ = heisenberg_hamiltonian(legs, length, 1.0, ns)   # fully polarised
        assert H.shape == (1, 1)
        assert abs(H[0, 0] - len(bonds(legs, length)) / 4) < 1e-14
    assert len(bonds(2, 6)) == 16


def test_heisenberg_ring_spectrum():
    # 4-site ring: spectrum of J S.S around the ring = {-2, -1, -1, -1, 0 (x7...), 1 (x5)}
    ev = []
    for nup in range(5):
        H, _ = heisenberg_hamiltonian(2, 2, 1.0, nup)
        ev.extend(np.linalg.eigvalsh(H.toarray()))
    ev = np.sort(np.round(ev, 12))
    vals, counts = np.unique(ev, return_counts=True)
    # singlet -2 (1), triplet -1 (3), singlet 0 (1) + 2 triplets 0 (6)... multiplicities sum 16
    assert counts.sum() == 16
    assert vals[0] == -2.0 and counts[0] == 1
    assert vals[-1] == 1.0 and counts[-1] == 5                 # the S=2 quintet
    assert vals[1] == -1.0 and counts[1] == 3


@pytest.mark.parametrize("legs,length", [(2, 3), (2, 4), (3, 3)])
def test_hubbard_symmetries(legs, length):
    U = 3.0
    ns = legs * length
    E = lambda a, b: ground_energy(hubbard_hamiltonian(legs, length, 1.0, U, a, b)[0])[0]
    # spin flip
    assert abs(E(ns // 2, ns // 2 - 1) - E(ns // 2 - 1, ns // 2)) < 1e-10
    # particle-hole on a bipartite lattice
    a, b = ns // 2 - 1, ns // 2 - 2
    assert abs(E(ns - a, ns - b) - (E(a, b) + U * (ns - a - b))) < 1e-9


def test_hermitian_and_conserving():
    H, basis = hubbard_hamiltonian(2, 3, 1.0, 2.0, 3, 2)
    assert abs(H - H.T).max() == 0.0
    H, basis = heisenberg_hamiltonian(3, 3, 1.0, 4)
    assert abs(H - H.T).max() == 0.0


def test_lieb_mattis_singlet():
    # bipartite ladders with equal sublattices: ground state is a singlet, so the
    # S_z=0 ground energy is strictly below the S_z=1 one
    for legs, length in [(2, 4), (2, 6)]:
        ns = legs * length
        e0 = ground_energy(heisenberg_hamiltonian(legs, length, 1.0, ns // 2)[0])[0]
        e1 = ground_energy(heisenberg_hamiltonian(legs, length, 1.0, ns // 2 + 1)[0])[0]
        assert e0 < e1 - 1e-6
    e0 = ground_energy(hubbard_hamiltonian(2, 3, 1.0, 4.0, 3, 3)[0])[0]
    e1 = ground_energy(hubbard_hamiltonian(2, 3, 1.0, 4.0, 4, 2)[0])[0]
    assert e0 < e1 - 1e-6


def test_full_fock_kron_construction_agrees():
    """Brute force by a different route: Jordan-Wigner matrices over the full Fock
    space of a 2x2 Hubbard plaquette, restricted afterwards to a sector."""
    nm = 8
    I2 = np.eye(2); Z = np.diag([1.0, -1.0]); a = np.array([[0.0, 1.0], [0.0, 0.0]])  # |1> -> |0>

    def ann(j):
        # mode j is bit j; kron puts bit 0 last (fastest) -> build high bits first
        ops = [I2] * nm
        for k in range(j):
            ops[k] = Z
        ops[j] = a
        M = np.array([[1.0]])
        for k in reversed(range(nm)):
            M = np.kron(M, ops[k])
        return M

    c = [ann(j) for j in range(nm)]
    U, t = 2.5, 1.0
    H = np.zeros((2 ** nm, 2 ** nm))
    for (i, j) in bonds(2, 2):
        for s in range(2):
            H -= t * (c[2 * i + s].T @ c[2 * j + s] + c[2 * j + s].T @ c[2 * i + s])
    for i in range(4):
        H += U * (c[2 * i].T @ c[2 * i]) @ (c[2 * i + 1].T @ c[2 * i + 1])
    Hs, basis = hubbard_hamiltonian(2, 2, t, U, 2, 1)
    assert np.allclose(Hs.toarray(), H[np.ix_(basis, basis)], atol=1e-14)


def test_oracle_lanczos_vs_eigh():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((300, 300)); A = A + A.T
    th, x, info = lanczos_ground(lambda v: A @ v, rng.standard_normal(300), max_iter=300, tol=1e-15)
    ev, evec = np.linalg.eigh(A)
    assert abs(th - ev[0]) < 1e-10 * abs(ev[0])
    assert abs(abs(x @ evec[:, 0]) - 1) < 1e-8
    H, _ = heisenberg_hamiltonian(2, 6, 1.0, 6)
    th, x, info = lanczos_ground(lambda v: H @ v, rng.standard_normal(H.shape[0]), tol=1e-15)
    assert abs(th - np.linalg.eigvalsh(H.toarray())[0]) < 1e-12
