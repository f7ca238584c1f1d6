"""Online stage of Polar Express in FP64 (test infrastructure, see package doc).

The iteration of eq. (iteration) with the odd quintic of Section 3.5:
    A = X X^T,  B = b A + c A^2,  X <- a X + B X,
formed on the smaller side of X (the Gram matrix is min(m,n) square; for a
tall input the iteration runs on G^T and the result is transposed back, which
is the same polynomial applied to the same singular values).

Normalisation (Appendix A.1 listing, the form used for every GPU result):
    X_0 = G / (1.01 ||G||_F + 1e-7)
or, with ``norm_mode=1``, Algorithm 1's  X_0 = G / (||G||_F + 1e-2).

Inputs are converted exactly to float64; all arithmetic is float64.
"""
from __future__ import annotations

import numpy as np


def normalise(G: np.ndarray, norm_mode: int = 0) -> np.ndarray:
    """X_0 from G (Appendix A.1 listing; Algorithm 1 when norm_mode == 1)."""
    G = np.asarray(G, dtype=np.float64)
    fro = float(np.sqrt(np.sum(G * G)))
    if norm_mode == 0:
        return G / (1.01 * fro + 1e-7)
    if norm_mode == 1:
        return G / (fro + 1e-2)
    raise ValueError("norm_mode must be 0 or 1")


def polar_express(G: np.ndarray, abc, norm_mode: int = 0, return_steps: bool = False):
    """X_T for an m x n input G with per-step coefficients ``abc`` (T x 3)."""
    G = np.asarray(G, dtype=np.float64)
    if G.ndim != 2:
        raise ValueError("G must be 2-D")
    abc = np.asarray(abc, dtype=np.float64).reshape(-1, 3)
    m, n = G.shape
    if m == 0 or n == 0:
        return np.zeros((m, n))
    tall = m > n
    X = normalise(G.T if tall else G, norm_mode)
    steps = []
    for a, b, c in abc:
        A = X @ X.T
        B = b * A + c * (A @ A)
        X = a * X + B @ X
        if return_steps:
            steps.append(X.T.copy() if tall else X.copy())
    out = X.T if tall else X
    if return_steps:
        return out, steps
    return out


def rel_fro(X: np.ndarray, ref: np.ndarray) -> float:
    """||X - ref||_F / ||ref||_F in float64 (the parity metric)."""
    X = np.asarray(X, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.linalg.norm(ref))
    num = float(np.linalg.norm(X - ref))
    return num / den if den > 0 else num
