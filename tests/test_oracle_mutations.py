"""Planted mistakes in copies of the oracle's arithmetic must fail its pins.

Each mutant is a plausible slip (a dropped term, a sign, a transposed operand,
a wrong index, a wrong normalisation); the test asserts that the pin used for
the real oracle rejects it.  Mistakes are planted here on the CPU only.
"""
import numpy as np

import synth
from oracle import schedule as S
from oracle import spectral as SP

ABC5 = S.greedy_schedule(1e-3, 5).abc


def _iterate(G, abc, mutant):
    X = G / (1.01 * np.linalg.norm(G) + 1e-7)
    if mutant == "bad_norm":
        X = G / (np.linalg.norm(G) + 1e-7)
    for a, b, c in abc:
        A = X.T @ X if mutant == "gram_wrong_side" else X @ X.T
        if mutant == "drop_c":
            B = b * A
        elif mutant == "sign_b":
            B = -b * A + c * A @ A
        elif mutant == "swap_bc":
            B = c * A + b * A @ A
        else:
            B = b * A + c * A @ A
        if mutant == "right_multiply":
            X = a * X + X @ B.T
        else:
            X = a * X + B @ X
    return X


def _appendix_c_pin(iterate, m=30, n=50):
    r = synth.rng(101)
    G = synth.usv(r, m, n, synth.spectrum_loguniform(r, min(m, n), 1e-3, 1.0))
    with np.errstate(all="ignore"):
        X = iterate(G.G)
    if not np.all(np.isfinite(X)) or np.abs(X).max() > 1e6:
        return False
    err = SP.spec_norm(X - G.polar())
    pred = SP.predicted_polar_error(SP.normalised_spectrum(G.sigma), ABC5)
    return abs(err - pred) <= 1e-12 * max(1, pred)


def test_correct_iteration_passes():
    assert _appendix_c_pin(lambda G: _iterate(G, ABC5, None))


def test_mutants_fail():
    for mutant in ("bad_norm", "drop_c", "sign_b", "swap_bc"):
        assert not _appendix_c_pin(lambda G: _iterate(G, ABC5, mutant)), mutant
    # operand-order slips only show on a square input, where they conform
    assert _appendix_c_pin(lambda G: _iterate(G, ABC5, None), 40, 40)
    for mutant in ("gram_wrong_side", "right_multiply"):
        assert not _appendix_c_pin(lambda G: _iterate(G, ABC5, mutant), 40, 40), mutant


def test_schedule_mutants_fail_table_pin(golden_dir):
    """A recentring from the cushioned end instead of l_t, or a safety factor
    applied before the bound update, both move the printed table."""
    import os
    paper = np.loadtxt(os.path.join(golden_dir, "paper_coeffs_ell1e-3.txt"))
    good = S.greedy_schedule(1e-3, 6, safety=1.0).abc_unsafe
    assert np.max(np.abs(good - paper[:6]) / np.abs(paper[:6])) <= 1e-13
    # mutant 1: no re-centring
    bad1 = S.greedy_schedule(1e-3, 6, safety=1.0, recentre=False).abc_unsafe
    assert np.max(np.abs(bad1 - paper[:6]) / np.abs(paper[:6])) > 1e-6
    # mutant 2: Algorithm 1's u/10 cushion
    bad2 = S.greedy_schedule(1e-3, 6, safety=1.0, tenth_rule=True).abc_unsafe
    assert np.max(np.abs(bad2 - paper[:6]) / np.abs(paper[:6])) > 1e-6
    # mutant 3: wrong initial trial points (swapped weights) converge to the
    # same optimum -- the exchange is self-correcting, so the table pin cannot
    # and need not catch it; the equioscillation pin checks the optimum itself.
