"""Spectrum-aware initialisation for matrices with a large outlying singular
value, in FP64 (test infrastructure, see package doc).

Appendix "Initialization for Matrices with Large Spectral Gaps", the case k = 1:
* a lower bound z <= sigma_1 from the power method (subspace iteration with
  one vector) on the Gram matrix A = X X^T of the normalised input;
* the Frobenius identity ||X||_F^2 = sum_j sigma_j^2 then bounds the rest of
  the spectrum: sigma_2, ..., sigma_n <= w = sqrt(||X||_F^2 - z^2);
* when the two ranges are apart (z > w), the odd cubic p(x) = a x + b x^3
  with p(w) = 1 and p(z) = 1 (eq. init_poly) is applied once,
  X <- a X + b A X, before the ordinary schedule.

Readings: eq. (init_poly) is printed for ||X||_F = 1; here X is
normalised as for the ordinary iteration (Appendix A.1 listing), so the
interpolation conditions are used with F = ||X||_F, which gives
a = (z^2 + z w + w^2) / (z w (z + w)), b = -1 / (z w (z + w)) (the printed
formula at F = 1).  The power method starts from a fixed sign vector (below)
and runs ``iters`` steps; z = sqrt(||A v||) for the last unit vector v, a lower
bound on sigma_1 since ||A v|| <= ||A||_2 = sigma_1^2.  When z <= w the step
is skipped (p = identity).
"""
from __future__ import annotations

import numpy as np

from .iteration import normalise


def start_vector(s: int) -> np.ndarray:
    """v_i = +-1/sqrt(s), the sign from bit 31 of Knuth's multiplicative hash
    (i * 2654435761) mod 2^32 of the index i (a counter-based sequence both
    sides compute from this definition)."""
    i = np.arange(s, dtype=np.uint64)
    h = (i * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)
    sign = np.where(h & np.uint64(0x80000000), -1.0, 1.0)
    return sign / np.sqrt(s)


def power_lower_bound(A: np.ndarray, iters: int) -> float:
    """z = sqrt(||A v_{k-1}||) after ``iters`` power steps v <- A v / ||A v||
    from ``start_vector``: a lower bound on sigma_1(X) for A = X X^T."""
    v = start_vector(A.shape[0])
    nrm = 0.0
    for _ in range(iters):
        y = A @ v
        nrm = float(np.linalg.norm(y))
        if nrm == 0.0:
            return 0.0
        v = y / nrm
    return float(np.sqrt(nrm))


def init_coefficients(z: float, F: float):
    """(a, b) of the cubic through (w, 1) and (z, 1), w = sqrt(F^2 - z^2);
    (1, 0) when z <= w (no separated outlier)."""
    w2 = F * F - z * z
    if not (z > 0.0) or w2 <= 0.0:
        return 1.0, 0.0
    w = float(np.sqrt(w2))
    if z <= w:
        return 1.0, 0.0
    den = z * w * (z + w)
    return (z * z + z * w + w * w) / den, -1.0 / den


def spectrum_aware_polar_express(G, abc, iters: int = 16, norm_mode: int = 0):
    """The initialisation step followed by the ordinary iteration with ``abc``."""
    G = np.asarray(G, dtype=np.float64)
    m, n = G.shape
    if m == 0 or n == 0:
        return np.zeros((m, n))
    tall = m > n
    X = normalise(G.T if tall else G, norm_mode)
    A = X @ X.T
    z = power_lower_bound(A, iters)
    a, b = init_coefficients(z, float(np.sqrt(np.trace(A))))
    X = a * X + b * (A @ X)
    for a_, b_, c_ in np.asarray(abc, dtype=np.float64).reshape(-1, 3):
        A = X @ X.T
        X = a_ * X + (b_ * A + c_ * (A @ A)) @ X
    return X.T if tall else X
