"""Pins of the oracle's Muon step (Section 1.1) against the definitions it
writes out: the momentum recursion unrolled over several steps equals its
closed form, beta = 0 reduces to the gradient, the weight step moves W by
exactly -lr polar(M) (plus the decoupled decay), and the direction is the
oracle's Polar Express of M itself."""
import numpy as np

import synth
from oracle import iteration as OI
from oracle import muon as MU
from oracle import schedule as OS


def test_momentum_closed_form():
    r = synth.rng(91)
    abc = OS.greedy_schedule(1e-3, 5).abc
    Gs = [r.standard_normal((20, 50)) for _ in range(4)]
    M = np.zeros((20, 50))
    W = r.standard_normal((20, 50))
    beta = 0.9
    for G in Gs:
        M, X, W = MU.muon_step(G, M, W, abc, lr=0.01, beta=beta)
    closed = sum((1 - beta) * beta ** (len(Gs) - 1 - k) * G for k, G in enumerate(Gs))
    assert np.allclose(M, closed, rtol=1e-14, atol=1e-15)


def test_beta_zero_and_weight_step():
    r = synth.rng(92)
    abc = OS.greedy_schedule(1e-3, 5).abc
    G = r.standard_normal((30, 12))
    M0 = r.standard_normal((30, 12))
    W0 = r.standard_normal((30, 12))
    M, X, W = MU.muon_step(G, M0, W0, abc, lr=0.05, beta=0.0)
    assert np.array_equal(M, G)
    assert np.allclose(X, OI.polar_express(G, abc), rtol=0, atol=0)
    assert np.allclose(W, W0 - 0.05 * X, rtol=0, atol=1e-15)
    _, X2, W2 = MU.muon_step(G, M0, W0, abc, lr=0.05, beta=0.0, wd=0.1)
    assert np.allclose(W2, (1 - 0.005) * W0 - 0.05 * X2, rtol=0, atol=1e-15)


def test_step_direction_is_nearly_orthogonal():
    """With enough steps and a well-conditioned momentum, the step direction
    is the polar factor: its singular values are 1 to the schedule's error."""
    r = synth.rng(93)
    S = synth.usv(r, 40, 90, np.linspace(1.0, 0.2, 40))
    abc = OS.greedy_schedule(1e-3, 8).abc
    _, X, _ = MU.muon_step(S.G, np.zeros_like(S.G), np.zeros_like(S.G), abc, lr=1.0, beta=0.0)
    sv = np.linalg.svd(X, compute_uv=False)
    assert np.max(np.abs(sv - 1.0)) <= 1e-2
    assert np.linalg.norm(X - S.polar(), 2) <= 1e-2
