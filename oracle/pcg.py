"""Algorithm 1 (PCGM) for Delta delta~ = r_delta with preconditioner P
(Sec. III), and plain CG (P = I).

    r = r_delta - Delta delta^(0);  d = P^-1 r;  mu = d' r
    loop:
        y = Delta d
        theta = mu / (y' d)
        delta += theta d
        r     -= theta y
        stop test
        q = P^-1 r;  mu' = q' r
        d = q + (mu'/mu) d;  mu = mu'

Readings:
  * The printed direction update reads d = r + (mu'/mu) d; the preconditioned
    CG of the cited source (and the only form that converges to the solution
    with a non-identity P) is d = q + (mu'/mu) d.  The printed r_theta in the
    initial residual is read as r_delta.
  * Stop test: the paper stops on ||r||_inf < eps (absolute).  Here the test
    is the relative 2-norm ||r||_2 <= tol * ||r_delta||_2 (relative to the
    right-hand side, not to r^(0), so a warm start is judged against the same
    target), confirmed by recomputing the true residual r_delta - Delta delta;
    if the true residual fails, PCG restarts from it (d = P^-1 r).
  * max_iter is not given by the paper; default 10000.
Vectors may have any shape; dot products are taken over all entries.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return float(np.vdot(a, b))


def pcg(apply_A, apply_Pinv, b, x0=None, tol=1e-10, max_iter=10000,
        keep_iterates=False):
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.sqrt(_dot(b, b))
    r = b - apply_A(x)
    hist = dict(res=[np.sqrt(_dot(r, r)) / bnorm], iterates=[], restarts=0,
                alpha=[], beta=[])
    if keep_iterates:
        hist["iterates"].append(x.copy())
    if np.sqrt(_dot(r, r)) <= tol * bnorm:
        return x, 0, hist
    d = apply_Pinv(r)
    mu = _dot(d, r)
    it = 0
    while it < max_iter:
        y = apply_A(d)
        theta = mu / _dot(y, d)
        x = x + theta * d
        r = r - theta * y
        it += 1
        hist["alpha"].append(theta)
        rn = np.sqrt(_dot(r, r))
        hist["res"].append(rn / bnorm)
        if keep_iterates:
            hist["iterates"].append(x.copy())
        if rn <= tol * bnorm:
            r_true = b - apply_A(x)
            if np.sqrt(_dot(r_true, r_true)) <= tol * bnorm:
                break
            hist["restarts"] += 1
            r = r_true
            d = apply_Pinv(r)
            mu = _dot(d, r)
            continue
        q = apply_Pinv(r)
        mu_new = _dot(q, r)
        beta = mu_new / mu
        hist["beta"].append(beta)
        d = q + beta * d
        mu = mu_new
    return x, it, hist


def cg(apply_A, b, **kw):
    return pcg(apply_A, lambda r: r.copy(), b, **kw)
