"""Pins of the oracle's spectrum-aware initialisation (appendix on matrices
with large spectral gaps, k = 1):

* the interpolating cubic written as this oracle derives it (general F)
  agrees with the form eq. (init_poly) prints for F = 1;
* p(w) = p(z) = 1, p(x) >= x / w on [0, w] (the paper's argument), and
  p(1) > 1/sqrt(2) over the valid range of z (stated in the paper);
* the power-method value is a lower bound on sigma_1 and converges to it for
  a separated outlier;
* on a diagonal input the whole method reduces to the scalar maps (init
  cubic, then the schedule's composite) on the diagonal;
* for a separated outlier (32 x 32, sigma = (1, 0.02/j)) the init step in
  place of one ordinary step leaves a several times smaller polar error.
"""
import numpy as np
import pytest

import synth
from oracle import iteration as OI
from oracle import schedule as OS
from oracle import spectral_init as SI


@pytest.mark.parametrize("z", [0.71, 0.8, 0.9, 0.99, 0.999])
def test_coefficients_match_printed_form(z):
    w = np.sqrt(1 - z * z)
    a, b = SI.init_coefficients(z, 1.0)
    a_p = (z * z * (z + w) - w) / (z * w * (2 * z * z - 1))
    b_p = (w - z) / (z * w * (2 * z * z - 1))
    assert abs(a - a_p) <= 1e-12 * abs(a_p) and abs(b - b_p) <= 1e-12 * abs(b_p)


@pytest.mark.parametrize("F", [1.0, 1 / 1.01, 0.5])
def test_interpolation_and_shape(F):
    for zr in [0.72, 0.85, 0.97, 0.999]:
        z = zr * F
        w = np.sqrt(F * F - z * z)
        a, b = SI.init_coefficients(z, F)
        p = lambda x: a * x + b * x ** 3
        assert abs(p(w) - 1) <= 1e-12 and abs(p(z) - 1) <= 1e-12
        x = np.linspace(0, w, 1001)
        assert np.all(p(x) >= x / w - 1e-12)
        if F == 1.0:
            assert p(1.0) > 1 / np.sqrt(2)
    # no separated outlier: identity
    assert SI.init_coefficients(0.6, 1.0) == (1.0, 0.0)


def test_power_lower_bound():
    r = synth.rng(95)
    S = synth.usv(r, 60, 150, np.r_[1.0, 0.05 * np.ones(59)])
    X = S.G / np.linalg.norm(S.G)
    A = X @ X.T
    s1 = np.linalg.norm(X, 2)
    for k in (1, 2, 4, 16):
        z = SI.power_lower_bound(A, k)
        assert z <= s1 * (1 + 1e-15)
    assert abs(SI.power_lower_bound(A, 16) - s1) <= 1e-10
    # Gaussian: still a lower bound
    G = r.standard_normal((40, 90))
    X = G / np.linalg.norm(G)
    assert SI.power_lower_bound(X @ X.T, 3) <= np.linalg.norm(X, 2)


def test_start_vector_definition():
    v = SI.start_vector(8)
    h = [(i * 2654435761) % 2 ** 32 for i in range(8)]
    assert np.array_equal(np.sign(v), [-1.0 if x & 0x80000000 else 1.0 for x in h])
    assert abs(np.linalg.norm(v) - 1) <= 1e-15


def test_diagonal_input_reduces_to_scalar_maps():
    sig = np.array([1.0, 0.02, 0.01, 5e-3, 1e-3])
    G = np.zeros((5, 9))
    G[np.arange(5), np.arange(5)] = sig
    abc = OS.greedy_schedule(1e-3, 5).abc
    X = SI.spectrum_aware_polar_express(G, abc, iters=30)
    sh = sig / (1.01 * np.linalg.norm(sig) + 1e-7)
    z = SI.power_lower_bound(np.diag(sh ** 2), 30)
    a, b = SI.init_coefficients(z, float(np.linalg.norm(sh)))
    expect = OS.composite(abc, a * sh + b * sh ** 3)
    assert np.allclose(np.diag(X[:, :5]), expect, rtol=1e-12, atol=1e-15)
    assert np.count_nonzero(X[:, 5:]) == 0


def test_outlier_spectrum_converges_faster():
    """The appendix's point: for a separated outlier the init step makes more
    progress than an ordinary step.  sigma = (1, 0.02/j for j = 2..32): with
    the init step in place of the first of 7 ordinary steps the polar error is
    several times smaller (the tail is lifted by ~1/w at once)."""
    r = synth.rng(96)
    S = synth.usv(r, 32, 32, np.r_[1.0, 0.02 / np.arange(2, 33)])
    P = S.polar()
    abc = OS.greedy_schedule(1e-3, 7).abc
    plain = np.linalg.norm(OI.polar_express(S.G, abc) - P, 2)
    init = np.linalg.norm(SI.spectrum_aware_polar_express(S.G, abc[:6]) - P, 2)
    assert init < 0.5 * plain
