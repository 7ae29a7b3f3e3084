"""Local observables of a superblock state (test infrastructure).

The paper's stripe analysis (Eqs. (2)-(4)) uses, for the site in column x and
leg y (1-based in the paper, 0-based here),

* the hole density            h(x, y) = 1 - <n_{x,y,up} + n_{x,y,dn}>,
* the staggered spin density  s(x, y) = <n_{x,y,up} - n_{x,y,dn}>,
* its leg maximum             S(x) = max_y |s(x, y)|,

with <.> the ground-state expectation value.  For the spin model a site has
one spin: n_up = 1/2 + S^z, n_dn = 1/2 - S^z, so h = 0 and s = 2 <S^z>.

A superblock state fixes these exactly on its two explicit columns (column 2
at lattice column ``ncols(block 1)``, column 3 right after it): the density
operators of a column are diagonal in its occupation basis, so

    <n_{y,sigma}> = sum over packed slots |psi|^2 * (bit (y, sigma) of i2 or i3).

Plain sums in float64; the bit layout is that of ``oracle.local``.
"""
from __future__ import annotations

import numpy as np

from .superblock import Superblock


def _occupations(model, states: np.ndarray) -> np.ndarray:
    """(len(states), legs, 2) occupations n_{y,sigma} of column states."""
    b = np.asarray(states, dtype=np.int64)[:, None]
    y = np.arange(model.legs)[None, :]
    if model.fermionic:
        up = (b >> (2 * y)) & 1
        dn = (b >> (2 * y + 1)) & 1
    else:
        up = (b >> y) & 1
        dn = 1 - up
    return np.stack([up, dn], axis=-1).astype(np.float64)


def column_densities(sb: Superblock, psi: np.ndarray) -> np.ndarray:
    """<n_{x,y,sigma}> on the superblock's two explicit columns.

    Returns an array (2, legs, 2): [column 2 or 3][leg][spin up, down], for
    a unit-norm packed state ``psi``."""
    psi = np.asarray(psi, dtype=np.float64)
    _, i2, i3, _ = sb.indices_of_packed()
    p = psi * psi
    out = np.zeros((2, sb.model.legs, 2))
    for k, cols in enumerate((i2, i3)):
        occ = _occupations(sb.model, cols)
        out[k] = np.einsum("i,iys->ys", p, occ)
    return out


def hole_and_spin_density(n: np.ndarray):
    """h = 1 - (n_up + n_dn) and s = n_up - n_dn from densities (..., 2)."""
    n = np.asarray(n, dtype=np.float64)
    return 1.0 - n[..., 0] - n[..., 1], n[..., 0] - n[..., 1]


def staggered_max(s: np.ndarray) -> np.ndarray:
    """S(x) = max over legs of |s(x, y)| (last axis = legs)."""
    return np.max(np.abs(np.asarray(s, dtype=np.float64)), axis=-1)


def lattice_densities(model, length: int, basis: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """<n_{x,y,sigma}> of a lattice state (brute-force basis of ``oracle.lattice``):
    (length, legs, 2).  Site (x, y) is number x*legs + y; Hubbard mode 2*site + sigma."""
    p = np.asarray(psi, dtype=np.float64) ** 2
    b = np.asarray(basis, dtype=np.int64)
    out = np.zeros((length, model.legs, 2))
    for x in range(length):
        for y in range(model.legs):
            site = x * model.legs + y
            if model.fermionic:
                out[x, y, 0] = p @ ((b >> (2 * site)) & 1)
                out[x, y, 1] = p @ ((b >> (2 * site + 1)) & 1)
            else:
                up = (b >> site) & 1
                out[x, y, 0] = p @ up
                out[x, y, 1] = p @ (1 - up)
    return out
