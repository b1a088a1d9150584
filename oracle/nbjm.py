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

``nbjm_solve`` runs the nested iteration as a solver in its own right (the
paper's comparison method: the block Jacobi outer iteration of eq.
"outer_jacobi_iterations" with L inner sweeps of eq. "inner_iteration_NBJM")
until the relative residual ||r - Delta delta^(s)||_2 <= tol ||r||_2.
Readings:
  * Inner start.  With theta^(0) = 0 in every outer iteration (as printed,
    and as the preconditioner needs) the outer iteration is
    delta <- Upsilon_L (r + Xi~ delta), whose fixed point
    (Upsilon_L^-1 - Xi~)^-1 r is not Delta^-1 r for finite L.  The
    standalone solver therefore starts each inner iteration from the outer
    iterate, theta^(0) = delta^(s); then a fixed point satisfies
    Phi~ delta = r + Xi~ delta + Omega~ delta, i.e. Delta delta = r, and one
    outer step is delta <- G delta + Upsilon_L r with
    G = Upsilon_L Xi~ + (Phi~^-1 Omega~)^L.
  * Stop test.  The printed test on ||delta^(s+1) - delta^(s)||_inf is
    absolute and scale dependent; the residual test is the one Algorithm 1
    uses, so both solvers stop at the same accuracy.  The increment norm is
    recorded as well.
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


def nbjm_solve(r, delta_op, xi, omega, phi_solve, L: int, tol: float = 1e-10,
               max_sweeps: int = 100000):
    """Standalone NBJM (outer iteration to convergence, each inner iteration
    started from the outer iterate).  Returns the iterate,
    the number of outer sweeps, and the history of relative residuals and
    increment infinity norms (one entry per sweep)."""
    rn = np.linalg.norm(r)
    delta = np.zeros_like(r)
    hist = dict(res=[], inc=[])
    for s in range(1, max_sweeps + 1):
        r_theta = r + xi(delta)
        theta = delta                       # inner start: the outer iterate
        for _ in range(L):
            theta = phi_solve(r_theta + omega(theta))
        hist["inc"].append(float(np.abs(theta - delta).max()))
        delta = theta
        res = np.linalg.norm(r - delta_op(delta)) / rn
        hist["res"].append(float(res))
        if res <= tol:
            return delta, s, hist
    return delta, max_sweeps, hist


def slab_nbjm_solve(ops, L: int = 2, tol: float = 1e-10, max_sweeps: int = 100000):
    """nbjm_solve on ``slab.SlabOperators`` for Delta delta~ = r_delta."""
    return nbjm_solve(ops.r_delta(), ops.delta, ops.xi, ops.omega, ops.phi_solve, L,
                      tol, max_sweeps)
