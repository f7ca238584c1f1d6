"""Pins for the oracle's l-predictor pieces (oracle/mlp.py)."""
import numpy as np

import synth
from oracle import iteration as I
from oracle import mlp as M
from oracle import schedule as S
from oracle import spectral as SP


def test_moments_equal_traces_of_gram_powers():
    """tr(A^k) of A = X_0 X_0^T equals sum sigma_hat^(2k) (spectral theorem)."""
    r = synth.rng(3)
    G = synth.usv(r, 40, 90, synth.spectrum_loguniform(r, 40, 1e-3, 1.0))
    X0 = I.normalise(G.G)
    A = X0 @ X0.T
    A2 = A @ A
    traces = [np.trace(A), np.trace(A2), np.trace(A @ A2), np.trace(A2 @ A2)]
    m = M.moments_from_spectrum(SP.normalised_spectrum(G.sigma))
    assert np.allclose(traces, m, rtol=1e-12)
    # the entrywise forms the GPU accumulates
    assert np.isclose(np.sum(A * A), m[1], rtol=1e-12)
    assert np.isclose(np.sum(A * A2), m[2], rtol=1e-12)
    assert np.isclose(np.sum(A2 * A2), m[3], rtol=1e-12)


def test_features_are_scale_and_rotation_invariant_where_stated():
    """Features depend only on (s, L, spectrum): rotations of G leave them fixed."""
    r = synth.rng(4)
    G = synth.usv(r, 30, 50, synth.spectrum_powerlaw(30, 0.7))
    s1 = np.linalg.svd(I.normalise(G.G), compute_uv=False)
    Q = synth.haar(r, 30, 30)
    s2 = np.linalg.svd(I.normalise(Q @ G.G), compute_uv=False)
    f1 = M.features(30, 50, M.moments_from_spectrum(s1))
    f2 = M.features(30, 50, M.moments_from_spectrum(s2))
    assert np.allclose(f1, f2, atol=1e-10)
    # participation ratio bounds: 1 <= m1^2/m2 <= s, so feature 14 >= 0
    assert f1[14] >= -1e-12 and f1[9] >= -1e-12


def test_class_errors_match_matrix_iteration():
    """Appendix C: the label's per-class error equals ||X_T' - UV^T||_2 of the
    class's T'-step iteration."""
    r = synth.rng(5)
    G = synth.usv(r, 24, 48, synth.spectrum_loguniform(r, 24, 1e-4, 1.0))
    s_hat = SP.normalised_spectrum(G.sigma)
    errs = M.class_errors(s_hat, 5)
    steps = M.class_steps(5)
    for c in (0, 3, 4, 7):
        abc = S.greedy_schedule(M.CLASS_ELL[c], int(steps[c])).abc
        X = I.polar_express(G.G, abc)
        assert abs(SP.spec_norm(X - G.polar()) - errs[c]) <= 1e-10


def test_class_table():
    """Class 4 is the paper's fixed schedule for all T steps; the others pair
    an l with T' <= T; a class's T'-step schedule is the first T' steps of its
    T-step schedule (the construction is greedy)."""
    assert M.CLASS_TABLE[M.FIXED_CLASS] == (1e-3, None)
    st = M.class_steps(5)
    assert st[M.FIXED_CLASS] == 5 and np.all(st <= 5) and st.min() >= 1
    for (l, _), k in zip(M.CLASS_TABLE, st):
        assert np.array_equal(S.greedy_schedule(l, int(k)).abc, S.greedy_schedule(l, 5).abc[:k])
    assert np.array_equal(M.class_steps(3), np.minimum(st, 3))


def test_label_rule():
    """Fewest steps within the fixed class's error; then the smaller error."""
    steps = np.array([2, 3, 3, 4, 5, 4, 5, 5])
    errs = np.array([0.5, 0.2, 0.1, 0.05, 0.1, 0.03, 0.02, 0.01])
    assert M.label(errs, steps) == 2          # 3 steps, 0.1 <= 0.1
    errs2 = errs.copy(); errs2[4] = 0.04
    assert M.label(errs2, steps) == 5         # 4 steps: class 5 (0.03) beats class 3 (0.05 > 0.04)
    errs3 = errs.copy(); errs3[4] = 0.015
    assert M.label(errs3, steps) == 7         # only 5-step classes qualify; the smallest error


def test_gradient_matches_finite_differences():
    r = np.random.default_rng(6)
    theta = M.init_params(1) + 0.01 * r.standard_normal(M.N_PARAMS)
    X = r.standard_normal((9, M.N_IN))
    y = r.integers(0, M.N_OUT, 9)
    loss, g = M.loss_and_grad(theta, X, y)
    idx = r.choice(M.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (M.loss_and_grad(tp, X, y)[0] - M.loss_and_grad(tm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_and_convergence():
    """Bias-corrected Adam moves each coordinate by exactly lr on its first step
    and minimises a quadratic."""
    th = np.array([1.0, -2.0, 3.0])
    m = np.zeros(3); v = np.zeros(3)
    th1, m, v = M.adam(th, np.array([0.3, -5.0, 1e-3]), m, v, 1, 0.01)
    assert np.allclose(np.abs(th1 - th), 0.01, rtol=1e-4)
    th = np.array([4.0, -3.0]); m = np.zeros(2); v = np.zeros(2)
    for t in range(1, 3001):
        th, m, v = M.adam(th, 2 * th, m, v, t, 0.05)
    assert np.all(np.abs(th) < 1e-2)


def test_learning_signal_exists():
    """The best class depends on the spectrum: a slowly decaying spectrum needs
    fewer steps than the fixed schedule (a class of larger l with T' < T), a
    log-uniform one down to 1e-5 a smaller l over all T steps."""
    T = 5
    steps = M.class_steps(T)
    flat = SP.normalised_spectrum(np.linspace(1.0, 0.5, 500))
    wide = SP.normalised_spectrum(np.geomspace(1.0, 1e-5, 500))
    cf = M.label(M.class_errors(flat, T), steps)
    cw = M.label(M.class_errors(wide, T), steps)
    assert steps[cf] < T
    assert steps[cw] == T and M.CLASS_ELL[cw] < 1e-3
