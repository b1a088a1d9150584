"""Spectrum estimates from the coefficients of (P)CG (Sec. III: the
convergence rate of Algorithm 1 is set by the condition number of the
preconditioned operator; Sec. V compares kappa(Delta) with
kappa(P_S^-1/2 Delta P_S^-1/2)).

CG on A x = b (preconditioner P, Algorithm 1) is the Lanczos process on
P^-1 A in disguise: with the step lengths alpha_k (theta of Algorithm 1) and
the direction coefficients beta_k = mu_{k+1} / mu_k, the k x k symmetric
tridiagonal matrix

    T[0, 0]     = 1 / alpha_0
    T[j, j]     = 1 / alpha_j + beta_{j-1} / alpha_{j-1}       (j >= 1)
    T[j, j + 1] = T[j + 1, j] = sqrt(beta_j) / alpha_j

is the Lanczos matrix of P^-1 A (similar to P^-1/2 A P^-1/2) in the basis
of the normalised preconditioned residuals, so its extreme eigenvalues
converge to those of P^-1 A from inside the spectrum.  kappa is estimated
as lambda_max(T) / lambda_min(T).  The eigenvalues of T are taken with
LAPACK's symmetric tridiagonal solver (scipy ``eigvalsh_tridiagonal``).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def lanczos_matrix(alpha, beta):
    """Diagonal and off-diagonal of T from k step lengths and k - 1 (or more)
    direction coefficients."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    k = len(alpha)
    if k == 0:
        raise ValueError("no CG iterations")
    diag = 1.0 / alpha
    diag[1:] += beta[:k - 1] / alpha[:k - 1]
    off = np.sqrt(beta[:k - 1]) / alpha[:k - 1]
    return diag, off


def spectrum_estimate(alpha, beta):
    """(lambda_min, lambda_max, kappa) of T."""
    diag, off = lanczos_matrix(alpha, beta)
    ev = sla.eigvalsh_tridiagonal(diag, off) if len(diag) > 1 else diag.copy()
    lo, hi = float(ev.min()), float(ev.max())
    return lo, hi, hi / lo


def condition_from_cg(apply_A, apply_Pinv, b, tol=1e-10, max_iter=10000):
    """Runs Algorithm 1 from zero (``pcg.pcg``) and returns the estimate of
    the spectrum of P^-1 A from its coefficients, plus the iteration count."""
    from . import pcg
    _, it, hist = pcg.pcg(apply_A, apply_Pinv, b, tol=tol, max_iter=max_iter)
    lo, hi, kap = spectrum_estimate(hist["alpha"], hist["beta"])
    return dict(lambda_min=lo, lambda_max=hi, kappa=kap, iterations=it)
