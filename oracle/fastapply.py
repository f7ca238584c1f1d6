"""Fast polynomial iteration for rectangular matrices in FP64 (test
infrastructure, see package doc).

Appendix G ("Fast Polynomial Iteration for Rectangular Matrices"),
Algorithm 4: for odd polynomials p_t(x) = x h_t(x^2) the composite applied to
a matrix X with Gram matrix Y (formed on the smaller side) is X Q_T, where
    Q_0 = I,  R_t = Q_{t-1}^T Y Q_{t-1},  Q_t = Q_{t-1} h_t(R_t),
so only two rectangular products (Y and the final product) are needed for
any number of steps; here h_t(y) = a_t + b_t y + c_t y^2 in Horner form,
h_t(R) = a_t I + R (b_t I + c_t R).

Restarting (Appendix G): the iteration is applied to k steps at a time, the
next segment starting from X_k with a fresh Y; restarting after every step is
the ordinary iteration.  In the first segment Y is replaced by Y + eps I
(the paper's guard against spurious negative eigenvalues); in our
orientation Y = X X^T, and X Q becomes Q X (both are polynomials in Y).

Reading: the input is normalised as for the ordinary iteration
(Appendix A.1 listing, 1.01 ||G||_F + 1e-7); the paper's remark that its
fast-iteration runs normalised by ||X||_F + 1e-3 is not adopted, so that the
two paths are comparable.

Inputs are converted exactly to float64; all arithmetic is float64.
"""
from __future__ import annotations

import numpy as np

from .iteration import normalise


def fast_polar_express(G, abc, restart: int = 3, eps: float = 1e-3, norm_mode: int = 0):
    """X_T of Algorithm 4 with restarts every ``restart`` steps and the shift
    ``eps`` on the first segment's Gram matrix."""
    G = np.asarray(G, dtype=np.float64)
    if G.ndim != 2:
        raise ValueError("G must be 2-D")
    if restart < 1:
        raise ValueError("restart must be >= 1")
    abc = np.asarray(abc, dtype=np.float64).reshape(-1, 3)
    m, n = G.shape
    if m == 0 or n == 0:
        return np.zeros((m, n))
    tall = m > n
    X = normalise(G.T if tall else G, norm_mode)
    s = X.shape[0]
    eye = np.eye(s)
    t, first = 0, True
    while t < abc.shape[0]:
        k = min(restart, abc.shape[0] - t)
        Y = X @ X.T
        if first and eps:
            Y = Y + eps * eye
        Q = eye
        for a, b, c in abc[t:t + k]:
            R = Q.T @ Y @ Q
            Q = Q @ (a * eye + R @ (b * eye + c * R))
        X = Q @ X
        t += k
        first = False
    return X.T if tall else X


def fast_scalar_map(sigma, abc, restart: int = 3, eps: float = 1e-3):
    """What Algorithm 4 with restarts does to one singular value sigma of the
    normalised X: each segment multiplies sigma by q(y) = phi(sqrt(y)) / sqrt(y)
    at y = sigma^2 (+ eps in the first segment), phi the segment's composite."""
    x = np.asarray(sigma, dtype=np.float64).copy()
    abc = np.asarray(abc, dtype=np.float64).reshape(-1, 3)
    t, first = 0, True
    while t < abc.shape[0]:
        k = min(restart, abc.shape[0] - t)
        r = np.sqrt(x * x + (eps if first else 0.0))
        y = r.copy()
        for a, b, c in abc[t:t + k]:
            z = y * y
            y = y * (a + z * (b + c * z))
        x = x * np.where(r > 0, y / np.where(r > 0, r, 1.0), np.prod(abc[t:t + k, 0]))
        t += k
        first = False
    return x
