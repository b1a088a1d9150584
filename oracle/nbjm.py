"""Algorithm 2 (NBJM) run for a fixed number of sweeps, used as the
preconditioner of Algorithm 1 (Sec. IV, "Positive-definiteness of
Preconditioner" and Theorem 2).

    delta^(0) = 0
    for s = 0..S-1:
        r_theta^(s) = r + Xi~ delta^(s)
        theta^(0) = 0
        for l = 0..L-1:
            theta^(l+1) = Phi~^-1 (r_theta^(s) + Omega~ theta^(l))
        delta^(s+1) = theta^(L)
    return delta^(S)

Readings: the printed algorithm never assigns delta^(s+1); it is theta^(L)
(this is what the proof of Theorem 2 iterates).  The early exit on
||delta^(s+1) - delta^(s)|| is not taken: Theorem 2 describes exactly S outer
sweeps, and a preconditioner that changes from call to call would break PCG.
Theorem 2 requires an even L for positive definiteness; this oracle accepts
any L >= 1 so that tests can also probe the closed form at L = 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def nbjm_apply(r, xi, omega, phi_solve, S: int, L: int):
    """Generic form on any vector representation supporting +, zeros_like."""
    delta = np.zeros_like(r)
    for _ in range(S):
        r_theta = r + xi(delta)
        theta = np.zeros_like(r)
        for _ in range(L):
            theta = phi_solve(r_theta + omega(theta))
        delta = theta
    return delta


def sparse_preconditioner(spl: dict, S: int, L: int):
    """P^-1 r for the explicit U x U splittings of ``splitting.splittings``;
    Phi~^-1 via a sparse LU factorisation (scipy splu)."""
    lu = spla.splu(spl["Phi"].tocsc())
    Xi, Om = spl["Xi"], spl["Omega"]
    return lambda r: nbjm_apply(r, lambda x: Xi @ x, lambda x: Om @ x,
                                lu.solve, S, L)


def slab_preconditioner(ops, S: int, L: int):
    """P^-1 r for ``slab.SlabOperators`` (vectors of shape (T+1, KNn))."""
    return lambda r: nbjm_apply(r, ops.xi, ops.omega, ops.phi_solve, S, L)
