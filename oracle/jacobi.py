"""Exact polar factor by a one-sided (Hestenes) Jacobi SVD in FP64
(test infrastructure, see package doc).

Target: polar(M) = U V^T for the reduced SVD M = U Sigma V^T, eq. (matrixsign).

One-sided Jacobi: for an m x n matrix W with m >= n, repeatedly rotate pairs of
columns (p, q) so that they become orthogonal; the accumulated rotations form
V and, at convergence, the columns of W V are U Sigma.  Pairs are visited in
round-robin (tournament) order, n/2 disjoint pairs per round, n-1 rounds per
sweep; sweeps stop when every pair satisfies
    |w_p . w_q| <= m * eps * ||w_p|| ||w_q||.
Rotation for a pair (alpha = ||w_p||^2, beta = ||w_q||^2, gamma = w_p . w_q):
    zeta = (beta - alpha) / (2 gamma), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
    c = 1 / sqrt(1 + t^2), s = c t,
    w_p <- c w_p - s w_q,  w_q <- s w_p + c w_q.
"""
from __future__ import annotations

import numpy as np

EPS = np.finfo(np.float64).eps


def _round_robin_pairs(n: int):
    """Tournament schedule: n-1 rounds (n even) of n/2 disjoint pairs."""
    idx = list(range(n))
    rounds = []
    for _ in range(n - 1):
        half = n // 2
        rounds.append((np.array(idx[:half]), np.array(idx[half:][::-1])))
        idx = [idx[0]] + [idx[-1]] + idx[1:-1]
    return rounds


def jacobi_svd(M: np.ndarray, max_sweeps: int = 60):
    """Reduced SVD of M (m x n) as (U, sigma, V) with M = U diag(sigma) V^T.

    sigma is sorted in decreasing order.  Columns of U for zero singular values
    are left as zero vectors (the polar factor is then only defined on the range).
    """
    M = np.asarray(M, dtype=np.float64)
    m, n = M.shape
    if m < n:
        U, s, V = jacobi_svd(M.T, max_sweeps)
        return V, s, U
    pad = n % 2
    W = np.concatenate([M, np.zeros((m, pad))], axis=1) if pad else M.copy()
    nn = n + pad
    V = np.eye(nn)
    rounds = _round_robin_pairs(nn)
    tol = m * EPS
    for _ in range(max_sweeps):
        worst = 0.0
        for P, Q in rounds:
            wp, wq = W[:, P], W[:, Q]
            alpha = np.einsum("ij,ij->j", wp, wp)
            beta = np.einsum("ij,ij->j", wq, wq)
            gamma = np.einsum("ij,ij->j", wp, wq)
            scale = np.sqrt(alpha * beta)
            off = np.zeros_like(gamma)
            nz = scale > 0
            off[nz] = np.abs(gamma[nz]) / scale[nz]
            worst = max(worst, float(off.max(initial=0.0)))
            act = off > tol
            if not np.any(act):
                continue
            zeta = np.zeros_like(gamma)
            zeta[act] = (beta[act] - alpha[act]) / (2.0 * gamma[act])
            t = np.zeros_like(gamma)
            t[act] = np.sign(zeta[act]) / (np.abs(zeta[act]) + np.sqrt(1.0 + zeta[act] ** 2))
            t[act & (zeta == 0)] = 1.0
            c = 1.0 / np.sqrt(1.0 + t * t)
            s = c * t
            vp, vq = V[:, P], V[:, Q]
            W[:, P] = c * wp - s * wq
            W[:, Q] = s * wp + c * wq
            V[:, P] = c * vp - s * vq
            V[:, Q] = s * vp + c * vq
        if worst <= tol:
            break
    W, V = W[:, :n], V[:n, :n] if not pad else V[:n, :n]
    sigma = np.sqrt(np.einsum("ij,ij->j", W, W))
    order = np.argsort(-sigma, kind="stable")
    sigma = sigma[order]
    W = W[:, order]
    V = V[:, order]
    U = np.zeros_like(W)
    nz = sigma > 0
    U[:, nz] = W[:, nz] / sigma[nz]
    return U, sigma, V


def polar_jacobi(M: np.ndarray) -> np.ndarray:
    """polar(M) = U V^T from ``jacobi_svd`` (eq. matrixsign)."""
    U, s, V = jacobi_svd(M)
    return U @ V.T


def polar_2x2(M: np.ndarray) -> np.ndarray:
    """Closed form for 2x2 (orthogonal Procrustes): polar(M) is the orthogonal
    Q maximising tr(Q^T M).  Rotations R(th) give tr = (p+s)cos th + (r-q) sin th,
    maximised at th = atan2(r-q, p+s) with value hypot(p+s, r-q); reflections
    F(th) = [[cos, sin],[sin, -cos]] give (p-s)cos th + (q+r) sin th, maximised at
    atan2(q+r, p-s) with value hypot(p-s, q+r)."""
    (p, q), (r, s) = np.asarray(M, dtype=np.float64)
    rot = np.hypot(p + s, r - q)
    ref = np.hypot(p - s, q + r)
    if rot >= ref:
        th = np.arctan2(r - q, p + s)
        return np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    th = np.arctan2(q + r, p - s)
    return np.array([[np.cos(th), np.sin(th)], [np.sin(th), -np.cos(th)]])
