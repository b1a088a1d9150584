"""Brute-force solution of the KKT system by a dense symmetric LDL'
factorisation (Sec. II-B, eq. "kkt_conditions").

The symmetric KKT system of the stacked QP (eq. "t_stacked_LQ_problem") with
multiplier lambda is

    [ Q~   0   A~' ] [x]   [  0     ]
    [ 0    R~  B~' ] [u] = [  0     ]
    [ A~   B~  0   ] [l]   [ r_delta]

Reading of the sign convention: the paper's Schur-complement solve uses
x~ = Q~^-1 A~' delta~ and Delta delta~ = r_delta, i.e. Q~ x~ - A~' delta~ = 0;
the printed KKT block has a "+".  The primal pair (x~, u~) does not depend on
the sign; the multiplier of the Schur-complement convention is
delta~ = -lambda, and that is what this module returns.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import stack


def kkt_matrix(p, S=None) -> np.ndarray:
    S = stack.stacked(p) if S is None else S
    At, Bt, Qt, Rt = S["At"], S["Bt"], S["Qt"], S["Rt"]
    nx, nu = At.shape[1], Bt.shape[1]
    Z = sp.csr_matrix((nx, nu))
    M = sp.bmat([[Qt, Z, At.T], [Z.T, Rt, Bt.T], [At, Bt, None]], format="csr")
    return M.toarray()


def ldl_solve(M: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve M z = b with the Bunch-Kaufman factorisation M = Lu D Lu'
    (scipy.linalg.ldl); Lu[perm] is unit lower triangular."""
    lu, d, perm = sla.ldl(M, lower=True)
    L = lu[perm]
    y = sla.solve_triangular(L, b[perm], lower=True, unit_diagonal=True)
    w = np.linalg.solve(d, y)          # d: 1x1 / 2x2 block diagonal
    v = sla.solve_triangular(L.T, w, lower=False, unit_diagonal=True)
    z = np.empty_like(v)
    z[perm] = v
    return z


def solve_kkt(p) -> dict:
    """Returns x~, u~ and delta~ (Schur-complement sign), all FP64."""
    S = stack.stacked(p)
    M = kkt_matrix(p, S)
    nx, nu = S["At"].shape[1], S["Bt"].shape[1]
    b = np.concatenate([np.zeros(nx), np.zeros(nu), S["r_delta"]])
    z = ldl_solve(M, b)
    x, u, lam = z[:nx], z[nx:nx + nu], z[nx + nu:]
    return dict(x=x, u=u, delta=-lam, residual=np.linalg.norm(M @ z - b))


def solve_schur_dense(p) -> np.ndarray:
    """delta~ = Delta^-1 r_delta by a dense Cholesky factorisation of Delta
    (Delta is positive definite, Sec. II-B)."""
    D = stack.delta_matrix(p).toarray()
    c = sla.cho_factor(D, lower=True)
    return sla.cho_solve(c, stack.r_delta(p))
