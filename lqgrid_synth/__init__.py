"""Seeded synthetic LQ-over-a-2D-grid problems.

This module only draws inputs.  It holds none of the solver's arithmetic and is
the one piece of code shared by the CPU oracle (``oracle/``) and the GPU path
(tests and ``bench.py`` feed its arrays to both).

Problem statement (Zafar & Manchester, Sec. II, eq. "2d_graph_dynamics" and the
LQ problem that follows it): K x N sub-systems, node (i, j) with i the vertical
(row) index in 1..K and j the horizontal (column) index in 1..N, evolve as

    x_{i,j,t+1} = A x_{i,j,t} + B u_{i,j,t} + E x_{i,j-1,t} + F x_{i,j+1,t}
                  + G x_{i-1,j,t} + H x_{i+1,j,t}

with stage cost x'Qx + u'Ru (t < T), terminal cost x'Q_T x, x_{i,j,0} = gamma.

Array layout (0-based, column index j outermost as in the paper's stacking
x_hat_t = col_j col_i x_{i,j,t}):

    A      [N][K][n][n]
    A_nbr  [N][K][4][n][n]   slot 0: E (from (i, j-1)), 1: F (from (i, j+1)),
                             2: G (from (i-1, j)),      3: H (from (i+1, j));
                             slots pointing off the grid are drawn but unused
    B      [N][K][n][m]
    Q, QT  [N][K][n][n]
    R      [N][K][m][m]
    x0     [N][K][n]

Recipe (all draws from numpy ``default_rng(seed)``, PCG64, in this order):
  1. A = standard_normal((N,K,n,n)); each node block is rescaled to spectral
     radius ``rho`` (a node whose spectral radius is exactly 0 is redrawn);
  2. A_nbr = cs * standard_normal((N,K,4,n,n));
  3. B = standard_normal((N,K,n,m));
  4. x0 = standard_normal((N,K,n)).
Q = QT = I_n, R = r_scale * I_m, zero spatial boundary states.

With ``weights="spd"`` (off by default, so the recipe above is unchanged) the
weights are instead drawn per node after x0, from the same generator:
  5. Q  = q_scale  * (M M' / n + I_n / 2),  M = standard_normal((N,K,n,n));
  6. QT = qt_scale * (M M' / n + I_n / 2),  a fresh M of the same shape;
  7. R  = r_scale  * (M M' / m + I_m / 2),  M = standard_normal((N,K,m,m)).
Each is symmetric positive definite (smallest eigenvalue >= scale / 2) and
differs from node to node, so a mix-up of the weights of two nodes (or of Q
and QT) changes the solution.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = ["Problem", "make_problem", "CONFIGS", "config_problem",
           "batched_dims", "batched_problems", "learned_problem"]


@dataclass
class Problem:
    K: int
    N: int
    T: int
    n: int
    m: int
    A: np.ndarray
    A_nbr: np.ndarray
    B: np.ndarray
    Q: np.ndarray
    R: np.ndarray
    QT: np.ndarray
    x0: np.ndarray
    seed: int = 0
    meta: dict = field(default_factory=dict)
    # spatial boundary states (Sec. II, eqs. "boundary_condition_i/j"), None
    # meaning zero: alpha_lo = x_{0,j,t} [T+1][N][n], alpha_hi = x_{K+1,j,t}
    # [T+1][N][n], beta_lo = x_{i,0,t} [T+1][K][n], beta_hi = x_{i,N+1,t}
    # [T+1][K][n] (0-based: the rows i = -1, i = K and the columns j = -1,
    # j = N next to the grid)
    alpha_lo: np.ndarray | None = None
    alpha_hi: np.ndarray | None = None
    beta_lo: np.ndarray | None = None
    beta_hi: np.ndarray | None = None
    # per-node state / input sizes (Sec. II), None meaning n and m everywhere
    n_node: np.ndarray | None = None
    m_node: np.ndarray | None = None
    # A, A_nbr, B, Q, R carry a leading time index t = 0..T-1
    time_varying: bool = False

    @property
    def has_boundary(self) -> bool:
        return any(b is not None for b in (self.alpha_lo, self.alpha_hi,
                                           self.beta_lo, self.beta_hi))

    @property
    def unknowns(self) -> int:
        """Number of PCG unknowns (entries of the multiplier vector)."""
        return self.K * self.N * self.n * (self.T + 1)


def _spectral_radius(M: np.ndarray) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(M))))


def make_problem(K: int, N: int, T: int, n: int, m: int, *, rho: float = 0.95,
                 cs: float = 0.1, seed: int = 0, r_scale: float = 0.1,
                 q_scale: float = 1.0, qt_scale: float | None = None,
                 weights: str = "identity", boundary: bool = False,
                 sizes: bool = False, time_varying: bool = False) -> Problem:
    """Draw one problem by the recipe in the module docstring.

    ``q_scale``/``qt_scale`` scale the weights; they exist so tests can
    exercise a terminal weight different from Q (default QT = Q).
    ``weights``: "identity" (the recipe's scaled identities) or "spd"
    (random per-node SPD weights, drawn after x0).  ``boundary``: draw
    non-zero spatial boundary states (standard normal, in the order
    alpha_lo, alpha_hi, beta_lo, beta_hi, after everything else).
    ``sizes``: heterogeneous sub-systems -- per-node n_node in U{1..n} and
    m_node in U{1..m} ([N][K] int arrays, drawn last); the arrays keep their
    padded shapes and the entries past a node's sizes hold the values drawn
    above, which a solver must ignore.
    ``time_varying``: A, A_nbr, B, Q and R get a leading time index t =
    0..T-1 (Sec. II: A_{i,j,t}, ...), each slice drawn as above in the same
    order (A rescaled per time and node); Q_T keeps none.  With "spd" weights
    every Q_t and R_t differs in t as well."""
    if min(K, N, T, n, m) < 1:
        raise ValueError("all dimensions must be >= 1")
    rng = np.random.default_rng(seed)
    if time_varying:
        return _make_tv(K, N, T, n, m, rho, cs, seed, r_scale, q_scale, qt_scale,
                        weights, boundary, sizes, rng)
    A = rng.standard_normal((N, K, n, n))
    sr_all = np.max(np.abs(np.linalg.eigvals(A)), axis=-1)
    if np.all(sr_all > 0.0):
        A *= (rho / sr_all)[..., None, None]
    else:  # a node to redraw: the same draws in node order
        for j in range(N):
            for i in range(K):
                sr = _spectral_radius(A[j, i])
                while sr == 0.0:
                    A[j, i] = rng.standard_normal((n, n))
                    sr = _spectral_radius(A[j, i])
                A[j, i] *= rho / sr
    A_nbr = cs * rng.standard_normal((N, K, 4, n, n))
    B = rng.standard_normal((N, K, n, m))
    x0 = rng.standard_normal((N, K, n))
    qt = q_scale if qt_scale is None else qt_scale
    if weights == "identity":
        eye_n = np.eye(n)
        Q = np.broadcast_to(q_scale * eye_n, (N, K, n, n)).copy()
        QT = np.broadcast_to(qt * eye_n, (N, K, n, n)).copy()
        R = np.broadcast_to(r_scale * np.eye(m), (N, K, m, m)).copy()
    elif weights == "spd":
        Q = q_scale * _random_spd(rng, N, K, n)
        QT = qt * _random_spd(rng, N, K, n)
        R = r_scale * _random_spd(rng, N, K, m)
    else:
        raise ValueError(f"unknown weights {weights!r}")
    p = Problem(K, N, T, n, m, A, A_nbr, B, Q, R, QT, x0, seed,
                dict(rho=rho, cs=cs, r_scale=r_scale, weights=weights))
    if boundary:
        p.alpha_lo = rng.standard_normal((T + 1, N, n))
        p.alpha_hi = rng.standard_normal((T + 1, N, n))
        p.beta_lo = rng.standard_normal((T + 1, K, n))
        p.beta_hi = rng.standard_normal((T + 1, K, n))
    if sizes:
        p.n_node = rng.integers(1, n + 1, size=(N, K)).astype(np.int32)
        p.m_node = rng.integers(1, m + 1, size=(N, K)).astype(np.int32)
    return p


def _make_tv(K, N, T, n, m, rho, cs, seed, r_scale, q_scale, qt_scale, weights,
             boundary, sizes, rng) -> Problem:
    """Time-varying data: the recipe with a leading time index on A, A_nbr,
    B (and on Q, R)."""
    A = rng.standard_normal((T, N, K, n, n))
    sr = np.max(np.abs(np.linalg.eigvals(A)), axis=-1)
    if not np.all(sr > 0.0):
        raise ValueError("a node block with spectral radius 0; use another seed")
    A *= (rho / sr)[..., None, None]
    A_nbr = cs * rng.standard_normal((T, N, K, 4, n, n))
    B = rng.standard_normal((T, N, K, n, m))
    x0 = rng.standard_normal((N, K, n))
    qt = q_scale if qt_scale is None else qt_scale
    if weights == "identity":
        Q = np.broadcast_to(q_scale * np.eye(n), (T, N, K, n, n)).copy()
        QT = np.broadcast_to(qt * np.eye(n), (N, K, n, n)).copy()
        R = np.broadcast_to(r_scale * np.eye(m), (T, N, K, m, m)).copy()
    elif weights == "spd":
        Q = q_scale * np.stack([_random_spd(rng, N, K, n) for _ in range(T)])
        QT = qt * _random_spd(rng, N, K, n)
        R = r_scale * np.stack([_random_spd(rng, N, K, m) for _ in range(T)])
    else:
        raise ValueError(f"unknown weights {weights!r}")
    p = Problem(K, N, T, n, m, A, A_nbr, B, Q, R, QT, x0, seed,
                dict(rho=rho, cs=cs, r_scale=r_scale, weights=weights, time_varying=True))
    p.time_varying = True
    if boundary:
        p.alpha_lo = rng.standard_normal((T + 1, N, n))
        p.alpha_hi = rng.standard_normal((T + 1, N, n))
        p.beta_lo = rng.standard_normal((T + 1, K, n))
        p.beta_hi = rng.standard_normal((T + 1, K, n))
    if sizes:
        p.n_node = rng.integers(1, n + 1, size=(N, K)).astype(np.int32)
        p.m_node = rng.integers(1, m + 1, size=(N, K)).astype(np.int32)
    return p


def _random_spd(rng, N: int, K: int, k: int) -> np.ndarray:
    """M M' / k + I / 2 per node, M standard normal (N, K, k, k)."""
    M = rng.standard_normal((N, K, k, k))
    S = np.einsum("jiab,jicb->jiac", M, M) / k + 0.5 * np.eye(k)
    return 0.5 * (S + np.swapaxes(S, -1, -2))


def redraw_x0(p: Problem, seed: int) -> np.ndarray:
    """A fresh initial state for the same dynamics (MPC-style re-solve)."""
    return np.random.default_rng(seed).standard_normal((p.N, p.K, p.n))


# The five workloads: tiny parity case, plain FP64 case, headline precision
# case, batched case, learned-warm-start case.
CONFIGS = {
    "tiny":    dict(K=4, N=4, T=20, n=2, m=1, rho=0.9, tol=1e-10),
    "plain":   dict(K=32, N=32, T=100, n=4, m=2, rho=0.95, tol=1e-10),
    "headline": dict(K=128, N=128, T=200, n=4, m=2, rho=0.95, tol=1e-8),
    "learned": dict(K=64, N=64, T=100, n=4, m=2, rho=0.95, tol=1e-8),
}


def config_problem(name: str, seed: int = 0) -> tuple[Problem, float]:
    c = dict(CONFIGS[name])
    tol = c.pop("tol")
    return make_problem(seed=seed, **c), tol


BATCHED_TOL = 1e-8  # tolerance of the batched workload


def batched_dims(P: int = 256, dims_seed: int = 999):
    """K, N ~ U{8..64}, T ~ U{50..200} drawn from default_rng(dims_seed)."""
    rng = np.random.default_rng(dims_seed)
    K = rng.integers(8, 65, size=P)
    N = rng.integers(8, 65, size=P)
    T = rng.integers(50, 201, size=P)
    return [(int(K[p]), int(N[p]), int(T[p])) for p in range(P)]


def batched_problems(P: int = 256, dims_seed: int = 999, seed0: int = 1000,
                     n: int = 4, m: int = 2, rho: float = 0.95):
    """Problem p uses seed seed0 + p."""
    return [make_problem(K, N, T, n, m, rho=rho, seed=seed0 + p)
            for p, (K, N, T) in enumerate(batched_dims(P, dims_seed))]


def learned_problem(seed: int) -> Problem:
    c = dict(CONFIGS["learned"])
    c.pop("tol")
    return make_problem(seed=seed, **c)
