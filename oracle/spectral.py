"""Spectral-norm error measures (test infrastructure, see package doc).

* ``spec_norm``: ||D||_2 as the square root of the largest eigenvalue of the
  smaller Gram matrix (symmetric eigensolver, FP64).
* ``spec_norm_power``: the same by power iteration on D^T D, for sizes where an
  eigensolver is too slow; runs until the Rayleigh quotient stalls.
* ``predicted_polar_error``: Appendix C -- for X_T = p(M) with M = U S V^T,
  polar(M) - p(M) = U (I - p(S)) V^T, so ||polar(M) - X_T||_2 equals
  max_i |1 - p(sigma_i)| over the singular values of the normalised input.
"""
from __future__ import annotations

import numpy as np

from .schedule import composite


def spec_norm(D: np.ndarray) -> float:
    D = np.asarray(D, dtype=np.float64)
    if D.size == 0:
        return 0.0
    G = D @ D.T if D.shape[0] <= D.shape[1] else D.T @ D
    w = np.linalg.eigvalsh(G)
    return float(np.sqrt(max(w[-1], 0.0)))


def spec_norm_power(D: np.ndarray, iters: int = 500, tol: float = 1e-12, seed: int = 0) -> float:
    D = np.asarray(D, dtype=np.float64)
    if D.size == 0:
        return 0.0
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(D.shape[1])
    v /= np.linalg.norm(v)
    prev = 0.0
    lam = 0.0
    for _ in range(iters):
        w = D.T @ (D @ v)
        lam = float(np.linalg.norm(w))
        if lam == 0.0:
            return 0.0
        v = w / lam
        if abs(lam - prev) <= tol * lam:
            break
        prev = lam
    return float(np.sqrt(lam))


def predicted_polar_error(sigma_hat, abc) -> float:
    """max_i |1 - phi_T(sigma_i)| (Appendix C identity)."""
    s = np.asarray(sigma_hat, dtype=np.float64)
    return float(np.max(np.abs(1.0 - composite(abc, s))))


def normalised_spectrum(sigma, fro=None, norm_mode: int = 0):
    """Singular values after the normalisation of the online stage."""
    s = np.asarray(sigma, dtype=np.float64)
    if fro is None:
        fro = float(np.sqrt(np.sum(s * s)))
    if norm_mode == 0:
        return s / (1.01 * fro + 1e-7)
    return s / (fro + 1e-2)
