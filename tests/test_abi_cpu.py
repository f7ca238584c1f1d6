"""Host-side checks of the C ABI (no GPU): the library loads and exports every
entry point declared in include/pe.h, the host FP64 schedule matches the oracle
and the paper's table, and argument checks reject bad input before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2505_16932_amd as pe
from oracle import schedule as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "pe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pe_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = pe.lib()
    syms = _declared_symbols()
    assert "pe_polar" in syms and "pe_coeffs" in syms and "pe_polar_batched" in syms
    for name in syms:
        assert hasattr(L, name), name


def test_default_cushion_is_the_ratio_rule_root():
    """pe_coeffs derives its default cushion from Appendix F's ratio-1/10 rule
    (bisection); it agrees with the factor printed in the Appendix A.2 listing
    to the rounding level of the minimax error it bisects on."""
    o = pe.CoeffOpts()
    pe.lib().pe_coeff_opts_default(ctypes.byref(o))
    assert abs(o.cushion - 0.02407327424182761) <= 1e-16
    assert abs(o.cushion - S.CUSHION) <= 1e-16


def test_coeffs_match_oracle_and_paper(golden_dir):
    paper = np.loadtxt(os.path.join(golden_dir, "paper_coeffs_ell1e-3.txt"))
    c = pe.coeffs(1e-3, 8, safety=1.0)
    rel = np.abs(c.abc - paper) / np.abs(paper)
    assert rel[:6].max() <= 1e-13
    assert rel[6].max() <= 2e-10
    assert np.array_equal(c.abc[7], paper[7])
    o = S.greedy_schedule(1e-3, 8, safety=1.0)
    assert np.allclose(c.bounds[:, 0], o.ell, rtol=1e-12, atol=1e-15)
    assert np.allclose(c.bounds[:, 1], o.u, rtol=1e-12)
    assert abs(c.err_bound - o.err_bound) <= 1e-12
    assert list(c.iters) == list(o.remez_iters)


@pytest.mark.parametrize("ell,T", [(1e-3, 5), (1e-3, 6), (1e-2, 7), (1e-4, 10), (0.3, 3)])
def test_coeffs_safety_variants(ell, T):
    for kw in [dict(), dict(safety_on_last=False), dict(cushion=0.0), dict(cushion=-1.0)]:
        c = pe.coeffs(ell, T, **kw)
        o = S.greedy_schedule(ell, T, cushion=0.0 if kw.get("cushion") == 0.0 else S.CUSHION,
                              safety_on_last=kw.get("safety_on_last", True),
                              tenth_rule=kw.get("cushion") == -1.0)
        # two float64 exchanges agree to within the conditioning of each step's
        # 4x4 system, which grows without bound as l_t/u_t -> 1 (Appendix E)
        for t in range(T):
            if kw.get("cushion") == -1.0:
                lo = max(o.ell[t], o.u[t] / 10)
            else:
                lo = max(o.ell[t], (0.0 if kw.get("cushion") == 0.0 else S.CUSHION) * o.u[t])
            hi = o.u[t]
            pts = np.array([lo, 0.75 * lo + 0.25 * hi, 0.25 * lo + 0.75 * hi, hi])
            cond = np.linalg.cond(np.stack([pts, pts ** 3, pts ** 5, [1, -1, 1, -1]], 1))
            tol = max(1e-13, 100 * cond * np.finfo(float).eps) if np.isfinite(cond) else 1.0
            assert np.allclose(c.abc[t], o.abc[t], rtol=tol, atol=1e-14), (kw, t, tol)


def test_coeffs_invalid_arguments():
    L = pe.lib()
    abc = (ctypes.c_double * 30)()
    for ell, T in [(0.0, 5), (1.0, 5), (-1.0, 5), (1e-3, 0), (1e-3, 65), (float("nan"), 3)]:
        assert L.pe_coeffs(ell, T, None, abc, None, None, None) == 1
    assert L.pe_coeffs(1e-3, 5, None, None, None, None, None) == 1


def _opts(T=5, compute=1, fp8=0):
    abc = np.tile(np.array(S.NS5), (T, 1)).reshape(-1).copy()
    o = pe.Opts(T, abc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), compute, fp8, 0, 0, None, -1, 0.0,
                0, 0, 0.0, 0.0, 0.0, 0.0, 0)
    return o, abc


def test_workspace_and_argument_checks():
    L = pe.lib()
    o, keep = _opts()
    m = pe.Matrix(16, 32, 300, 200, 200, 200, 1, 1)
    n1 = L.pe_workspace_size(1, ctypes.byref(m), ctypes.byref(o))
    assert n1 > 0
    # padded to 256 x 384, bf16 path: X as FP32 master and two bf16 copies
    # (X_t and X_{t+1}); A and B in bf16
    assert n1 >= 256 * 384 * (4 + 2 + 2) + 256 * 256 * (2 + 2)
    bad = [pe.Matrix(16, 32, 300, 200, 100, 200, 1, 1),   # ldg < n
           pe.Matrix(0, 32, 300, 200, 200, 200, 1, 1),    # null G
           pe.Matrix(16, 32, -1, 200, 200, 200, 1, 1),    # negative m
           pe.Matrix(16, 32, 3, 2, 2, 2, 7, 1)]           # bad dtype
    for b in bad:
        assert L.pe_workspace_size(1, ctypes.byref(b), ctypes.byref(o)) == 0
        assert L.pe_polar(ctypes.byref(b), ctypes.byref(o), None, 0, None) == 1
    o2, keep2 = _opts(T=0)
    assert L.pe_polar(ctypes.byref(m), ctypes.byref(o2), None, 0, None) == 1
    # tile ids: 0 (library choice), 1 (128), 2 (256); anything else is rejected
    for t, ok in ((0, True), (1, True), (2, True), (3, False), (128, False), (256, False), (-1, False)):
        o3, keep3 = _opts()
        o3.tile = t
        assert (L.pe_workspace_size(1, ctypes.byref(m), ctypes.byref(o3)) > 0) == ok
        if not ok:
            assert L.pe_polar(ctypes.byref(m), ctypes.byref(o3), None, 0, None) == 1
    # workspace too small or misaligned: rejected before any launch
    assert L.pe_polar(ctypes.byref(m), ctypes.byref(o), None, 0, None) == 4
    assert L.pe_polar(ctypes.byref(m), ctypes.byref(o), ctypes.c_void_p(256), 16, None) == 4
    assert L.pe_polar(ctypes.byref(m), ctypes.byref(o), ctypes.c_void_p(257), n1, None) == 4
    # m = 0 is a valid no-op that needs no workspace and launches nothing
    z = pe.Matrix(0, 0, 0, 7, 7, 7, 1, 1)
    assert L.pe_polar(ctypes.byref(z), ctypes.byref(o), None, 0, None) == 0
    assert L.pe_polar_batched(0, None, ctypes.byref(o), None, 0, None) == 0
    assert L.pe_status_string(4) == b"workspace missing, too small or not 256-byte aligned"


def test_learned_features_match_oracle_definition():
    """The host feature code used for training (product side) and the oracle's
    definition agree (both restate the same 16 features)."""
    from oracle import mlp as OM
    from paper_2505_16932_amd import learned as PL
    r = np.random.default_rng(3)
    for _ in range(20):
        s, L = int(r.integers(2, 3000)), int(r.integers(2, 9000))
        m = np.sort(r.uniform(1e-9, 1.0, 4))[::-1] ** np.array([1, 2, 3, 4])
        assert np.allclose(PL.features(s, L, m), OM.features(s, L, m), rtol=1e-12, atol=1e-12)


def test_learned_labels_match_oracle():
    from oracle import mlp as OM
    from paper_2505_16932_amd import learned as PL
    F, Y, E = PL.build_dataset(40, seed=11, T=5)
    rng = np.random.Generator(np.random.PCG64(11))
    scheds = OM.class_schedules(5)
    for i in range(40):
        m, n, sig, _ = PL.sample_spectrum(rng)
        sh = sig / (1.01 * np.sqrt(np.sum(sig * sig)) + 1e-7)
        e = OM.class_errors(sh, 5, scheds)
        # the two schedule builders differ by up to ~1e-7 relative on the
        # near-degenerate steps of the larger-l schedules (4x4 conditioning)
        assert np.allclose(E[i], e, rtol=1e-6, atol=1e-8)
        # the label: fewest steps within the fixed class's error (the oracle's rule)
        steps = OM.class_steps(5)
        assert e[Y[i]] <= e[OM.FIXED_CLASS] * (1 + 1e-6) + 1e-8
        assert steps[Y[i]] == steps[OM.label(e, steps)]
        assert np.allclose(F[i], OM.features(min(m, n), max(m, n), OM.moments_from_spectrum(sh)),
                           rtol=1e-5, atol=1e-5)


def test_tile_table_drives_the_tile_choice(tmp_path):
    """An autotuned table entry (class and call regime) changes the padding
    (128 vs 256) and so the workspace size; malformed tables are rejected;
    unknown classes keep the built-in choice."""
    L = pe.lib()
    o, keep = _opts()
    m = pe.Matrix(16, 32, 600, 1000, 1000, 1000, 1, 1)
    cls = L.pe_shape_class(1, 600, 1000).decode()
    assert cls == "bf16_s1024_a4"
    t = tmp_path / "tab.txt"
    sizes = {}
    for tile in (1, 2):
        # a call below 3e12 FLOP per step looks up the class's _x1 regime
        t.write_text(f"# test\n{cls}_x1 {tile}  # comment\n{cls}_xN {3 - tile}\n")
        assert L.pe_tile_table_load(str(t).encode()) == 0
        sizes[tile] = L.pe_workspace_size(1, ctypes.byref(m), ctypes.byref(o))
    assert sizes[2] > sizes[1]
    t.write_text("bf16_s256_a1 2\n")
    assert L.pe_tile_table_load(str(t).encode()) == 0
    # 600 x 1000 is not in this table: built-in choice (s >= 512 but few tiles -> 128)
    assert L.pe_workspace_size(1, ctypes.byref(m), ctypes.byref(o)) == sizes[1]
    t.write_text("bf16_s256_a1 7\n")
    assert L.pe_tile_table_load(str(t).encode()) == 1
    assert L.pe_tile_table_load(b"/nonexistent/table") == 1
    # restore the shipped table (if any) for later tests
    import os
    shipped = os.path.join(os.path.dirname(pe.LIB_PATH), "tile_table.txt")
    t.write_text("# empty\n")
    assert L.pe_tile_table_load((shipped if os.path.exists(shipped) else str(t)).encode()) == 0


@pytest.mark.parametrize("ell,T", [(1e-3, 8), (1e-2, 6), (0.2, 4)])
def test_cubic_coeffs_match_oracle(ell, T):
    c = pe.coeffs_cubic(ell, T)
    o = S.greedy_schedule_cubic(ell, T)
    assert np.allclose(c.abc, o.abc, rtol=1e-13, atol=1e-15)
    assert np.all(c.abc[:, 2] == 0.0)
    assert np.allclose(c.bounds[:, 0], o.ell, rtol=1e-12)
    assert abs(c.err_bound - o.err_bound) <= 1e-12
    c1 = pe.coeffs_cubic(ell, T, safety=1.0)
    assert np.allclose(c1.abc, S.greedy_schedule_cubic(ell, T, safety=1.0).abc, rtol=1e-13)
