"""Pins for the oracle's online stage, exact polar factor and error measures.

Pinned against: the scalar reduction of the iteration on diagonal inputs
(Section 2: p(M) = U p(Sigma) V^T), orthogonal inputs, the Appendix C identity,
invariances of polar(.) and of the odd-polynomial iteration, LAPACK's SVD,
a brute-force 2x2 Procrustes search, and library spectral norms.
"""
import numpy as np
import pytest

import synth
from oracle import iteration as I
from oracle import jacobi as J
from oracle import schedule as S
from oracle import spectral as SP
from oracle import lowprec as LP

ABC5 = S.greedy_schedule(1e-3, 5).abc


def test_diagonal_reduces_to_scalar_map():
    """Section 2 notation: p(M) = U p(Sigma) V^T, so a diagonal input maps its
    diagonal through the scalar composite of the normalised values."""
    d = np.array([3.0, 1.0, 0.2, 1e-3, 4e-5])
    G = np.diag(d)
    X = I.polar_express(G, ABC5)
    sig_hat = d / (1.01 * np.linalg.norm(d) + 1e-7)
    assert np.allclose(np.diag(X), S.composite(ABC5, sig_hat), rtol=1e-13, atol=1e-15)
    assert np.allclose(X - np.diag(np.diag(X)), 0.0, atol=1e-15)
    # rectangular diagonal, both orientations
    Gw = np.zeros((3, 7))
    Gw[np.arange(3), np.arange(3)] = [2.0, 0.5, 0.01]
    for G2 in (Gw, Gw.T):
        X2 = I.polar_express(G2, ABC5)
        s_hat = np.array([2.0, 0.5, 0.01]) / (1.01 * np.sqrt(4 + 0.25 + 1e-4) + 1e-7)
        assert np.allclose(X2[np.arange(3), np.arange(3)], S.composite(ABC5, s_hat), rtol=1e-13)


def test_orthogonal_input_is_scaled():
    """A square orthogonal Q has all singular values equal, so X_T = phi_T(s) Q
    with s = 1 / (1.01 sqrt(n) + 1e-7); with Newton-Schulz steps on a normalised
    orthogonal input, Q is an exact fixed point (15/8 - 10/8 + 3/8 = 1)."""
    r = synth.rng(5)
    n = 17
    Q = synth.haar(r, n, n)
    X = I.polar_express(Q, ABC5)
    s = 1.0 / (1.01 * np.sqrt(n) + 1e-7)
    assert np.allclose(X, S.composite(ABC5, s) * Q, atol=1e-13)
    # fixed point under NS5 steps once the singular values are 1
    X1 = Q.copy()
    for _ in range(3):
        A = X1 @ X1.T
        X1 = 15 / 8 * X1 + (-10 / 8 * A + 3 / 8 * A @ A) @ X1
    assert np.allclose(X1, Q, atol=1e-13)


@pytest.mark.parametrize("shape", [(40, 40), (30, 70), (90, 25)])
def test_appendix_c_identity(shape):
    """Appendix C: ||polar(M) - p(M)||_2 = max_i |1 - p(sigma_i)|."""
    m, n = shape
    r = synth.rng(11 + m)
    sig = synth.spectrum_loguniform(r, min(m, n), 1e-3, 1.0) * 3.0
    G = synth.usv(r, m, n, sig)
    X = I.polar_express(G.G, ABC5)
    err = SP.spec_norm(X - G.polar())
    s_hat = SP.normalised_spectrum(G.sigma)
    pred = SP.predicted_polar_error(s_hat, ABC5)
    assert abs(err - pred) <= 1e-12 * max(1.0, pred)


def test_invariances():
    """polar(G^T) = polar(G)^T, polar(Q1 G Q2) = Q1 polar(G) Q2 and scale
    invariance hold for the odd-polynomial iteration too."""
    r = synth.rng(21)
    G = r.standard_normal((23, 41))
    X = I.polar_express(G, ABC5)
    assert np.allclose(I.polar_express(G.T, ABC5), X.T, atol=1e-12)
    Q1 = synth.haar(r, 23, 23)
    Q2 = synth.haar(r, 41, 41)
    assert np.allclose(I.polar_express(Q1 @ G @ Q2, ABC5), Q1 @ X @ Q2, atol=1e-11)
    assert np.allclose(I.polar_express(7.5 * G, ABC5), X, atol=1e-7)


def test_orientation_does_not_change_the_polynomial():
    """Section 3.5: X(aI + Y(bI + cY)) with Y = X^T X equals aX + (bA + cA^2)X
    with A = X X^T; the oracle forms the Gram on the smaller side."""
    r = synth.rng(22)
    G = r.standard_normal((15, 60))
    X = I.normalise(G)
    for a, b, c in ABC5:
        Y = X.T @ X
        X = X @ (a * np.eye(60) + Y @ (b * np.eye(60) + c * Y))
    assert np.allclose(I.polar_express(G, ABC5), X, atol=1e-12)


def test_zero_and_empty():
    """Appendix A.1 listing: the 1e-7 guard maps a zero matrix to zeros."""
    assert np.array_equal(I.polar_express(np.zeros((5, 8)), ABC5), np.zeros((5, 8)))
    assert I.polar_express(np.zeros((0, 8)), ABC5).shape == (0, 8)


def test_many_steps_converge_to_polar():
    """Theorem 2: with l below sigma_min the iterates converge to polar(M)."""
    r = synth.rng(23)
    G = synth.usv(r, 50, 80, np.linspace(1.0, 0.05, 50))
    abc = S.greedy_schedule(1e-3, 12).abc
    abc[-3:] = S.NS5  # finish without the safety factor so the limit is 1
    X = I.polar_express(G.G, abc)
    assert SP.spec_norm(X - G.polar()) <= 1e-9


@pytest.mark.parametrize("shape", [(8, 8), (13, 5), (6, 21), (64, 33), (7, 1)])
def test_jacobi_svd_vs_lapack(shape):
    r = synth.rng(31 + shape[0] * 7 + shape[1])
    M = r.standard_normal(shape)
    U, s, V = J.jacobi_svd(M)
    s_ref = np.linalg.svd(M, compute_uv=False)
    assert np.allclose(s, s_ref, rtol=1e-12, atol=1e-14)
    assert np.allclose((U * s) @ V.T, M, atol=1e-12)
    Ul, sl, Vlt = np.linalg.svd(M, full_matrices=False)
    assert np.allclose(J.polar_jacobi(M), Ul @ Vlt, atol=1e-10)


def test_jacobi_known_spectrum():
    r = synth.rng(41)
    G = synth.usv(r, 120, 60, synth.spectrum_powerlaw(60))
    assert np.allclose(J.polar_jacobi(G.G), G.polar(), atol=1e-10)


def test_polar_2x2_brute_force():
    """2x2 polar factor = the orthogonal Q maximising tr(Q^T M), found by a
    brute-force search over rotations and reflections."""
    r = synth.rng(51)
    th = np.linspace(-np.pi, np.pi, 200001)
    c, s = np.cos(th), np.sin(th)
    for _ in range(20):
        M = r.standard_normal((2, 2))
        (p, q), (rr, ss) = M
        rot = (p + ss) * c + (rr - q) * s
        ref = (p - ss) * c + (q + rr) * s
        best = max(rot.max(), ref.max())
        Q = J.polar_2x2(M)
        assert abs(np.trace(Q.T @ M) - best) <= 1e-8
        assert np.allclose(Q, J.polar_jacobi(M), atol=1e-10)
        # the iteration with many steps converges to the same factor
        if np.min(np.linalg.svd(M, compute_uv=False)) / np.max(np.linalg.svd(M, compute_uv=False)) > 0.01:
            abc = S.greedy_schedule(1e-3, 10, safety=1.0).abc
            assert np.allclose(I.polar_express(M, abc), Q, atol=1e-6)


def test_spectral_norms():
    r = synth.rng(61)
    for shape in [(10, 30), (40, 12), (25, 25)]:
        D = r.standard_normal(shape)
        ref = np.linalg.norm(D, 2)
        assert abs(SP.spec_norm(D) - ref) <= 1e-12 * ref
        assert abs(SP.spec_norm_power(D, iters=5000, tol=1e-15) - ref) <= 1e-6 * ref


def test_bf16_rounding_vs_torch():
    """RNE bfloat16 from its definition agrees with torch's cast."""
    import torch
    r = synth.rng(71)
    x = np.concatenate([r.standard_normal(20000) * 10.0 ** r.uniform(-30, 30, 20000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, 1e-40])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(LP.round_bf16(x), ref)


def test_e4m3_rounding_vs_torch():
    """RNE OCP e4m3 from its definition agrees with torch.float8_e4m3fn for
    in-range values; beyond 448 the quantiser saturates."""
    import torch
    r = synth.rng(72)
    x = np.concatenate([r.uniform(-448, 448, 20000), r.standard_normal(20000) * 1e-2,
                        r.standard_normal(2000) * 1e-3,
                        np.array([0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -10, 0.0625 * 1.0625])])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = LP.round_e4m3(x.astype(np.float32).astype(np.float64))
    assert np.array_equal(got, ref)
    codes_ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(LP.e4m3_code(x.astype(np.float32).astype(np.float64)), codes_ref)
    assert LP.round_e4m3(np.array([500.0, -1e6]))[0] == 448.0
    assert LP.round_e4m3(np.array([500.0, -1e6]))[1] == -448.0
