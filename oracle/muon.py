"""One Muon optimizer step in FP64 (test infrastructure, see package doc).

Section 1.1 (The Muon Method): with learning rate lr and momentum coefficient
beta,
    M_t = beta M_{t-1} + (1 - beta) G_t,      W_{t+1} = W_t - lr polar(M_t),
where polar(M) is approximated by Polar Express (the same iteration as
``iteration.polar_express``).  Weight decay: the paper's GPT-2 runs use weight
decay 0.1 without stating its form; the decoupled form
W_{t+1} = (1 - lr wd) W_t - lr polar(M_t) is this oracle's reading (wd = 0
gives the update of Section 1.1 exactly).
"""
from __future__ import annotations

import numpy as np

from .iteration import polar_express


def muon_step(G, M, W, abc, lr: float, beta: float = 0.9, wd: float = 0.0, norm_mode: int = 0):
    """Returns (M_t, X_T = Polar Express of M_t, W_{t+1})."""
    G = np.asarray(G, dtype=np.float64)
    M = beta * np.asarray(M, dtype=np.float64) + (1.0 - beta) * G
    X = polar_express(M, abc, norm_mode)
    W = (1.0 - lr * wd) * np.asarray(W, dtype=np.float64) - lr * X
    return M, X, W
