"""FP64 reference for the learned l-predictor (test infrastructure, see package doc).

The paper fixes l = 1e-3 because a good lower bound on sigma_min is hard to
get cheaply and a wrong guess only costs a few iterations (Section 3.3).  The
predictor picks one of eight precomputed schedules per matrix from moments of
the step-1 Gram matrix A = X_0 X_0^T:
    m_k = tr(A^k) = sum_i sigma_hat_i^(2k),  k = 1..4,
which the GPU path accumulates from A (k = 1, 2) and A^2 (k = 3, 4).  A class
is a pair (l, T'): the greedy schedule for l run for T' <= T steps (steps past
T' leave X as it is), so a matrix whose spectrum allows it finishes early.

* ``features``: the 16 inputs, from (s, L, m_1..m_4).
* ``moments_from_spectrum``: m_k from the normalised singular values.
* ``class_errors``: the Appendix C identity -- the polar error of class c is
  max_i |1 - phi^c(sigma_hat_i)| for its T'-step composite phi^c -- so labels
  need only the spectrum.
* ``label``: the class with the fewest steps whose error does not exceed the
  fixed class's (l = 1e-3, T steps); among those the smallest error.
* ``forward`` / ``backward`` / ``adam``: the MLP 16 -> 64 -> 64 -> 8 with ReLU
  hidden layers and softmax cross-entropy, in float64.

Parameter layout (flat, float): W1 [16 x 64] (row = input), b1 [64],
W2 [64 x 64], b2 [64], W3 [64 x 8], b3 [8]; 5768 values.
"""
from __future__ import annotations

import numpy as np

from .schedule import composite, greedy_schedule

# (l, T') per class; T' = None means the call's T.  Class 4 is the paper's
# choice, l = 1e-3 for all T steps.
CLASS_TABLE = [(1e-1, 2), (1e-1, 3), (3e-2, 3), (1e-2, 4), (1e-3, None), (3e-3, 4), (3e-4, None),
               (1e-4, None)]
CLASS_ELL = np.array([c[0] for c in CLASS_TABLE])
FIXED_CLASS = 4
N_IN, N_H, N_OUT = 16, 64, 8
SHAPES = [(N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, N_OUT), (N_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in parts])


def moments_from_spectrum(sigma_hat):
    s2 = np.asarray(sigma_hat, dtype=np.float64) ** 2
    return np.array([np.sum(s2), np.sum(s2 ** 2), np.sum(s2 ** 3), np.sum(s2 ** 4)])


def features(s, L, m):
    """16 scale-aware features of a matrix with Gram moments m = (m1, m2, m3, m4)."""
    m1, m2, m3, m4 = [max(float(x), 1e-300) for x in m]
    ls, lL = np.log(max(s, 1)), np.log(max(L, 1))
    lm1, lm2, lm3, lm4 = np.log(m1), np.log(m2), np.log(m3), np.log(m4)
    den = max(ls, 1e-3)
    return np.array([
        ls / 8.0, lL / 8.0, lL - ls,
        lm1, lm2 / 4.0, lm3 / 8.0, lm4 / 8.0,
        (2 * lm1 - lm2) / den,            # log participation ratio / log s
        (2 * lm2 - lm4) / den,            # second-order effective rank / log s
        lm1 + lm3 - 2 * lm2,              # spread of sigma^2 about its mean (>= 0)
        lm2 + lm4 - 2 * lm3,
        lm4 / 8.0 - lm1 / 2.0,            # tight sigma_max bound vs RMS scale
        (2 * lm1 - lm2) / 8.0,
        (2 * lm2 - lm4) / 8.0,
        ls - (2 * lm1 - lm2),             # log(s / participation ratio) >= 0
        1.0,
    ])


def class_steps(T):
    """T' of every class for a T-step call."""
    return np.array([min(T, k) if k is not None else T for _, k in CLASS_TABLE])


def class_schedules(T, safety=1.01):
    """Each class's T'-step greedy schedule (a list of (T', 3) arrays)."""
    return [greedy_schedule(float(l), int(k), safety=safety).abc
            for (l, _), k in zip(CLASS_TABLE, class_steps(T))]


def class_errors(sigma_hat, T, scheds=None):
    """Polar error of each class's schedule (Appendix C identity)."""
    scheds = scheds or class_schedules(T)
    x = np.asarray(sigma_hat, dtype=np.float64)
    return np.array([np.max(np.abs(1.0 - composite(abc, x))) for abc in scheds])


def label(errs, steps, rtol=1e-9):
    """Fewest steps among the classes whose error is within the fixed class's
    (rtol, plus 1e-15 absolute); ties to the smaller error, then the smaller
    index."""
    errs = np.asarray(errs)
    steps = np.asarray(steps)
    ok = np.flatnonzero(errs <= errs[FIXED_CLASS] * (1 + rtol) + 1e-15)
    fewest = steps[ok].min()
    cand = ok[steps[ok] == fewest]
    return int(cand[np.argmin(errs[cand])])


def forward(theta, X):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    logits = h2 @ W3 + b3
    return logits, (X, z1, h1, z2, h2)


def loss_and_grad(theta, X, y):
    """Mean softmax cross-entropy over the batch and its gradient."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    logits, (X, z1, h1, z2, h2) = forward(theta, X)
    B = X.shape[0]
    z = logits - logits.max(axis=1, keepdims=True)
    p = np.exp(z)
    p /= p.sum(axis=1, keepdims=True)
    y = np.asarray(y, dtype=np.int64)
    loss = float(-np.mean(np.log(p[np.arange(B), y])))
    d3 = p.copy()
    d3[np.arange(B), y] -= 1.0
    d3 /= B
    gW3 = h2.T @ d3
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3.T) * (z2 > 0)
    gW2 = h1.T @ d2
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2.T) * (z1 > 0)
    gW1 = X.T @ d1
    gb1 = d1.sum(axis=0)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba), step counted from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-normal weights, zero biases."""
    r = np.random.default_rng(seed)
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            parts.append(r.standard_normal(s) * np.sqrt(2.0 / s[0]))
        else:
            parts.append(np.zeros(s))
    return pack(parts)
