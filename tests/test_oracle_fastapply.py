"""Pins of the oracle's Algorithm 4 (Appendix G, fast polynomial iteration for
rectangular matrices) against what the paper and the mathematics fix:

* restarting after every step is the ordinary iteration (Appendix G says so);
* without the first-segment shift, any restart interval computes the same
  composite as the ordinary iteration (the derivation of Algorithm 4:
  R_t = r_t(X), Q_t = q_t(X), X Q_T = phi_T(X));
* with the shift eps, the singular vectors are unchanged and each singular
  value follows the scalar map sigma -> sigma q(sqrt(sigma^2 + eps)) per
  segment, checked against a LAPACK SVD of the normalised input;
* transposition commutes with the method.
"""
import numpy as np
import pytest

import synth
from oracle import fastapply as FA
from oracle import iteration as OI
from oracle import schedule as OS


def _inputs():
    r = synth.rng(71)
    return [
        synth.usv(r, 40, 140, synth.spectrum_loguniform(r, 40, 1e-2, 1.0)).G,
        synth.usv(r, 90, 30, synth.spectrum_powerlaw(30)).G,
        r.standard_normal((24, 96)),
    ]


@pytest.mark.parametrize("T", [3, 5, 7])
def test_restart_every_step_is_the_ordinary_iteration(T):
    abc = OS.greedy_schedule(1e-3, T).abc
    for G in _inputs():
        ref = OI.polar_express(G, abc)
        got = FA.fast_polar_express(G, abc, restart=1, eps=0.0)
        assert OI.rel_fro(got, ref) <= 1e-13


@pytest.mark.parametrize("restart", [2, 3, 5, 8])
def test_unshifted_fast_iteration_equals_ordinary_iteration(restart):
    """Well-conditioned inputs (sigma_min / sigma_max >= 1e-2), so that the
    accumulated Q stays moderate and float64 rounding stays near 1e-13."""
    abc = OS.greedy_schedule(1e-3, 8).abc
    for G in _inputs():
        ref = OI.polar_express(G, abc)
        got = FA.fast_polar_express(G, abc, restart=restart, eps=0.0)
        assert OI.rel_fro(got, ref) <= 1e-10, restart


@pytest.mark.parametrize("restart,eps", [(3, 1e-3), (2, 1e-3), (5, 1e-2), (3, 0.0)])
def test_shifted_fast_iteration_matches_svd_scalar_map(restart, eps):
    abc = OS.greedy_schedule(1e-3, 6).abc
    for G in _inputs():
        m, n = G.shape
        X0 = OI.normalise(G.T if m > n else G)
        U, sig, Vt = np.linalg.svd(X0, full_matrices=False)
        expect = (U * FA.fast_scalar_map(sig, abc, restart, eps)) @ Vt
        expect = expect.T if m > n else expect
        got = FA.fast_polar_express(G, abc, restart=restart, eps=eps)
        assert OI.rel_fro(got, expect) <= 1e-10


def test_shift_only_touches_the_first_segment():
    """A second segment without the shift: changing eps changes the result
    only through the first segment's scalar map."""
    abc = OS.greedy_schedule(1e-3, 6).abc
    sig = np.array([0.9, 0.3, 1e-2, 1e-4])
    a = FA.fast_scalar_map(sig, abc, 3, 1e-3)
    # by hand: first segment with the shift, second without
    y = np.sqrt(sig ** 2 + 1e-3)
    x = OS.composite(abc[:3], y) / y * sig
    x = OS.composite(abc[3:], x)
    assert np.allclose(a, x, rtol=1e-13, atol=0)


def test_transpose_commutes():
    abc = OS.greedy_schedule(1e-3, 5).abc
    G = _inputs()[0]
    a = FA.fast_polar_express(G, abc, 3, 1e-3)
    b = FA.fast_polar_express(G.T, abc, 3, 1e-3)
    assert np.allclose(a, b.T, rtol=0, atol=1e-14)
