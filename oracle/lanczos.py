"""Plain Lanczos for the lowest eigenpair (test infrastructure).

The paper's exact-diagonalisation routine ("HMED") finds the ground state of
the superblock Hamiltonian by repeated products ``Hv``; the eigensolver is
not named, Lanczos is the standard choice.  This version is the textbook
three-term recurrence with *full* reorthogonalisation (classical
Gram-Schmidt applied twice), all in float64, the tridiagonal matrix
diagonalised with LAPACK after every step.  It keeps every Krylov vector, so
it is meant for vectors of up to a few million entries.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal


def lanczos_ground(matvec, v0, max_iter=400, tol=1e-14, min_iter=5):
    """Lowest eigenvalue and unit eigenvector of the operator ``matvec``.

    Stops when the lowest Ritz value changes by less than ``tol*|theta|``
    between steps and the Ritz residual estimate ``|beta_k y_k|`` is below
    ``sqrt(tol)*|theta|``, or on breakdown (an invariant subspace).
    Returns ``(theta, x, info)``.
    """
    q = np.asarray(v0, dtype=np.float64).copy()
    nrm = np.linalg.norm(q)
    if not np.isfinite(nrm) or nrm == 0.0:
        raise ValueError("bad start vector")
    N = q.size
    kmax = min(max_iter, N)
    Q = np.empty((kmax, N))
    Q[0] = q / nrm
    alpha, beta = [], []
    theta_old = None
    theta, y = None, None
    for k in range(kmax):
        w = matvec(Q[k])
        a = float(Q[k] @ w)
        alpha.append(a)
        Qk = Q[: k + 1]
        for _ in range(2):                       # CGS, twice
            w = w - Qk.T @ (Qk @ w)
        b = float(np.linalg.norm(w))
        if k == 0:
            theta, y = alpha[0], np.ones(1)
        else:
            evals, evecs = eigh_tridiagonal(np.array(alpha), np.array(beta),
                                            select="i", select_range=(0, 0))
            theta, y = float(evals[0]), evecs[:, 0]
        res = abs(b * y[-1])
        if b <= 1e-14 * max(1.0, abs(theta)) or k + 1 == kmax:
            break
        if (theta_old is not None and k + 1 >= min_iter
                and abs(theta - theta_old) <= tol * abs(theta)
                and res <= np.sqrt(tol) * max(1.0, abs(theta))):
            break
        theta_old = theta
        beta.append(b)
        Q[k + 1] = w / b
    n_used = len(alpha)
    x = Q[:n_used].T @ y
    x /= np.linalg.norm(x)
    r = matvec(x) - theta * x
    return theta, x, {"iterations": n_used, "residual": float(np.linalg.norm(r))}


def ground_state(matvec, n, seed=0, v0=None, **kw):
    """Lanczos from a seeded N(0,1) start vector (or ``v0``)."""
    if v0 is None:
        v0 = np.random.default_rng(seed).standard_normal(n)
    return lanczos_ground(matvec, v0, **kw)


def ground_state_arpack(matvec, n, v0=None, tol=0.0, ncv=None):
    """Lowest eigenpair by ARPACK's implicitly restarted Lanczos (large vectors)."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    op = LinearOperator((n, n), matvec=matvec, dtype=np.float64)
    vals, vecs = eigsh(op, k=1, which="SA", tol=tol, v0=v0, ncv=ncv)
    x = vecs[:, 0]
    r = matvec(x) - vals[0] * x
    return float(vals[0]), x, {"residual": float(np.linalg.norm(r))}


def lowest_two_arpack(matvec, n, v0=None, tol=0.0, ncv=None):
    """The two lowest eigenpairs by ARPACK, with their residual norms.

    Returns ``(theta0, theta1, x0, rho0, rho1)``.  The second pair gives the
    gap needed by the Kato-Temple bound on the first (see ``kato_temple_lower``).
    """
    from scipy.sparse.linalg import LinearOperator, eigsh
    op = LinearOperator((n, n), matvec=matvec, dtype=np.float64)
    vals, vecs = eigsh(op, k=2, which="SA", tol=tol, v0=v0, ncv=ncv)
    order = np.argsort(vals)
    vals, vecs = vals[order], vecs[:, order]
    res = [float(np.linalg.norm(matvec(vecs[:, i]) - vals[i] * vecs[:, i])) for i in range(2)]
    return float(vals[0]), float(vals[1]), vecs[:, 0], res[0], res[1]


def kato_temple_lower(theta, rho, upper_gap_bound):
    """Kato-Temple lower bound on the lowest eigenvalue of a symmetric operator.

    For a unit vector with Rayleigh quotient ``theta`` and residual norm
    ``rho``, and any ``b`` with ``theta < b <= lambda_1`` (the second
    eigenvalue), ``lambda_0 >= theta - rho**2 / (b - theta)`` (Kato 1949,
    Temple 1928).  ``upper_gap_bound`` is such a ``b``; None if it is not
    above ``theta``.
    """
    if not upper_gap_bound > theta:
        return None
    return theta - rho * rho / (upper_gap_bound - theta)
