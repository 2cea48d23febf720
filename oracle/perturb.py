"""Stability enforcement above the CFL limit (Sec. III-A).  FP64, dense.
Test infrastructure only.

Condition (singular_limit): the reduced leapfrog is stable iff every singular
value of De~^{-1/2} K~ Dm~^{-1/2} is below 2/dt.  The perturbation clamps the
singular values at gamma * 2/dt (gamma = 0.9999 in Sec. V) and rebuilds
K~' = De~^{1/2} U S' W^T Dm~^{1/2}.  Square roots here are the symmetric
(principal) ones, from ``eigh``.
"""
from __future__ import annotations

import numpy as np


def sym_sqrt(D: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Principal square root (or its inverse) of a symmetric positive definite matrix."""
    w, Q = np.linalg.eigh(0.5 * (D + D.T))
    if np.any(w <= 0):
        raise np.linalg.LinAlgError("matrix is not positive definite")
    s = w ** (-0.5 if inverse else 0.5)
    return (Q * s) @ Q.T


def scaled_singular_values(De: np.ndarray, Dm: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Singular values sigma_i of De^{-1/2} K Dm^{-1/2} (eq. (singular_limit))."""
    A = sym_sqrt(De, True) @ K @ sym_sqrt(Dm, True)
    return np.linalg.svd(A, compute_uv=False)


def perturb(De: np.ndarray, Dm: np.ndarray, K: np.ndarray, dt: float, gamma: float = 0.9999):
    """Sec. III-A, steps 1-3.  Returns (K', n_clamped, sigma, sigma').

    sigma'_i = sigma_i if sigma_i < gamma 2/dt, else gamma 2/dt.
    """
    De_h, Dm_h = sym_sqrt(De), sym_sqrt(Dm)
    De_ih, Dm_ih = sym_sqrt(De, True), sym_sqrt(Dm, True)
    A = De_ih @ K @ Dm_ih
    U, s, Wt = np.linalg.svd(A, full_matrices=False)
    lim = gamma * 2.0 / dt
    s2 = np.where(s < lim, s, lim)
    n = int(np.sum(s >= lim))
    Kp = De_h @ (U * s2) @ Wt @ Dm_h
    return Kp, n, s, s2


def iteration_matrix(P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """G = P^{-1} Q, the one-step map of eq. (MNAform) (dense, tiny cases)."""
    return np.linalg.solve(P, Q)
