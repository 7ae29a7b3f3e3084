"""CPU FP64 oracle for the direct 2-D DMRG superblock product ``Hv``.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP library in ``paper_0707_0159_amd``.

What it computes (Yamada, Okumura, Machida, "Direct Extension of DMRG toward
2-Dimensional Quantum Lattice Systems"):

* ``lattice``     -- brute-force Heisenberg / Hubbard Hamiltonians on an
                     s-leg x L ladder in the occupation basis (global
                     Jordan-Wigner order), the plain definition every other
                     piece is checked against.
* ``local``       -- one column (rung of s sites) as a set of explicit matrices.
* ``blocks``      -- blocks grown column by column (Fig. 1a), their truncation
                     by the reduced density matrix (the DMF/DMD routines).
* ``superblock``  -- the four-block superblock Hamiltonian of Eq. (1), the
                     index maps that turn the superblock vector into the
                     matrices V and V_c, and ``Hv`` computed two ways: as one
                     explicit sparse matrix (mode X) and in the paper's
                     matrix form H_l V + V H_r^T + H_c V_c (mode F).
* ``lanczos``     -- plain Lanczos with full reorthogonalisation.
* ``dmrg``        -- the infinite-system growth that produces truncated blocks.

Precision: float64 throughout.  Quantum numbers are integer pairs
``(n_up, n_dn)``; for the spin model ``n_dn`` is always 0 and ``n_up`` counts
up spins.
"""
