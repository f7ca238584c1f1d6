"""The learned l-predictor on the GPU: the training kernels against the FP64
oracle (forward, gradient, Adam step), the selection inside a plan (features
from the step-1 Gram moments against the oracle's features of the spectrum, the
class against the oracle MLP), the fallback, and the gain of the trained
network over the fixed l = 1e-3 schedule."""
import numpy as np
import pytest

import synth
from oracle import mlp as OM
from oracle import schedule as OS
from oracle import spectral as SP
from tests.gpu_util import device_input, relf, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import paper_2505_16932_amd as pe
    pe.lib()
    return pe


def _rand_problem(seed, B):
    r = np.random.default_rng(seed)
    theta = OM.init_params(seed) + 0.05 * r.standard_normal(OM.N_PARAMS)
    X = r.standard_normal((B, OM.N_IN))
    X[:, -1] = 1.0
    y = r.integers(0, OM.N_OUT, B)
    return theta, X, y


def _t(x, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype or np.float32)).cuda()


def test_mlp_forward_matches_oracle(pe):
    theta, X, _ = _rand_problem(1, 300)
    got = pe.mlp_forward(_t(theta), _t(X)).cpu().numpy()
    ref, _ = OM.forward(theta.astype(np.float32).astype(np.float64), X.astype(np.float32))
    assert np.allclose(got, ref, rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("B", [64, 200, 1024])
def test_mlp_gradient_matches_oracle(pe, B):
    theta, X, y = _rand_problem(2 + B, B)
    loss, grad = pe.mlp_grad(_t(theta), _t(X), _t(y, np.int32))
    th32 = theta.astype(np.float32).astype(np.float64)
    l_ref, g_ref = OM.loss_and_grad(th32, X.astype(np.float32), y)
    g = grad.cpu().numpy()
    assert abs(float(loss.item()) - l_ref) <= 1e-5 * max(1, l_ref)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"[mlp] B={B} gradient rel err {rel:.2e}", flush=True)
    assert rel <= 1e-5
    # (the oracle's gradient itself is pinned to finite differences on the CPU)


def test_adam_step_matches_oracle(pe):
    import torch
    theta, X, y = _rand_problem(9, 256)
    params = _t(theta)
    tr = pe.MLPTrainer(params, 256)
    th = theta.astype(np.float32).astype(np.float64)
    m = np.zeros_like(th); v = np.zeros_like(th)
    for step in range(1, 4):
        tr.train_step(_t(X), _t(y, np.int32), 1e-3)
        _, g = OM.loss_and_grad(th, X.astype(np.float32), y)
        th, m, v = OM.adam(th, g, m, v, step, 1e-3)
    torch.cuda.synchronize()
    assert np.allclose(params.cpu().numpy(), th, rtol=1e-4, atol=2e-6)


def class_schedule(pe, c, abc4, T=5):
    """(T', abc) of schedule class c in a T-step call: class 4 is the caller's
    schedule, the others pe_coeffs(l_c, T')."""
    steps = int(OM.class_steps(T)[c])
    if c == OM.FIXED_CLASS:
        return T, abc4
    return steps, pe.coeffs(OM.CLASS_ELL[c], steps).abc


def _materialise(k, m, n, sig):
    import torch
    r = synth.rng(2000 + k)
    S = synth.usv(r, m, n, sig)
    G, vals = device_input(S.G, torch.bfloat16)
    return G, vals


@pytest.fixture(scope="module")
def trained(pe):
    """A predictor trained on the device from spectrum-level data (T = 5)."""
    from paper_2505_16932_amd import learned as PL
    F, Y, E = PL.build_dataset(16384, seed=101, T=5)
    params = PL.train(F, Y, epochs=25, batch=1024, lr=3e-3, seed=0)
    return params


def test_training_gain_over_fixed_ell(pe, trained):
    """On held-out spectra the chosen schedules leave a smaller polar error
    (Appendix C identity) than the fixed l = 1e-3 schedule."""
    from paper_2505_16932_amd import learned as PL
    F, Y, E = PL.build_dataset(4096, seed=202, T=5)
    res = PL.evaluate(trained, F, E, T=5, Y=Y)
    print(f"[learned] held-out: mean steps {res['mean_steps']:.3f} of 5 (fewer on "
          f"{res['frac_fewer_steps']:.1%}); mean error fixed {res['mean_fixed']:.4f} chosen "
          f"{res['mean_chosen']:.4f}; worse on {res['frac_worse']:.1%} (mean excess "
          f"{res['mean_excess_when_worse']:.4f}); accuracy {res['accuracy']:.1%}", flush=True)
    assert res["mean_steps"] < 4.7
    assert res["mean_chosen"] <= res["mean_fixed"] * 1.02
    assert res["frac_worse"] <= 0.1


def test_selection_in_plan_matches_oracle(pe, trained):
    """Matrices with known spectra: GPU features from the step-1 Gram moments vs
    the oracle's features of the normalised spectrum; the class vs the oracle MLP
    on the GPU's features; the result vs a plain call with that class's schedule
    (split-K off on both sides, so that the two sum in the same order)."""
    import torch
    cases = [(300, 900, np.geomspace(1, 1e-5, 300)), (512, 512, synth.spectrum_powerlaw(512, 0.5)),
             (640, 200, np.linspace(1.0, 0.4, 200)), (256, 1536, synth.spectrum_powerlaw(256, 1.5))]
    Gs, vals = [], []
    for k, (m, n, sig) in enumerate(cases):
        g, v = _materialise(k, m, n, sig)
        Gs.append(g)
        vals.append(v)
    abc4 = OS.greedy_schedule(1e-3, 5).abc
    plan = pe.Plan(Gs, T=5, abc=abc4, compute="bf16", predictor=trained, out_dtype=torch.float32,
                   split_k=1)
    plan.launch(graph=False)
    torch.cuda.synchronize()
    cls, feats, est, flags = plan.selection()
    theta = trained.cpu().numpy().astype(np.float64)
    for k, v in enumerate(vals):
        s_hat = np.linalg.svd(v / (1.01 * np.linalg.norm(v) + 1e-7), compute_uv=False)
        m_, n_ = v.shape
        f_ref = OM.features(min(m_, n_), max(m_, n_), OM.moments_from_spectrum(s_hat))
        err = np.abs(feats[k] - f_ref)
        print(f"[learned] case {k}: class {cls[k]} max feature err {err.max():.2e}", flush=True)
        assert err.max() <= 2e-2
        logits, _ = OM.forward(theta, feats[k:k + 1].astype(np.float64))
        assert int(np.argmax(logits[0])) == cls[k]
        Tc, abcc = class_schedule(pe, int(cls[k]), abc4)
        Y = pe.polar(Gs[k], T=Tc, abc=abcc, compute="bf16", out_dtype=torch.float32, split_k=1)
        torch.cuda.synchronize()
        assert relf(to_np(plan.outs[k]), to_np(Y)) <= 1e-6
    plan.close()


def test_learned_plan_large_tile_split_k(pe):
    """The learned path on the 256 tile (8 waves): a 256 x 1024 matrix keeps the
    raw A^2 epilogue and its moment reduction in the GEMM kernel (no split of
    A^2), a 512 x 1024 matrix splits its Gram product, and a 2048 x 2048 matrix
    splits both, so its raw A^2 epilogue and moment reduction run in the
    split-K reduce kernel.
    Results equal the plain calls with the forced class's schedule; features
    agree with the oracle's features of the normalised spectrum."""
    import torch
    cases = [(256, 1024, synth.spectrum_powerlaw(256, 1.0)), (512, 1024, np.geomspace(1, 1e-3, 512)),
             (2048, 2048, synth.spectrum_powerlaw(2048, 0.7))]
    Gs, vals = [], []
    for k, (m, n, sig) in enumerate(cases):
        g, v = _materialise(30 + k, m, n, sig)
        Gs.append(g)
        vals.append(v)
    abc4 = OS.greedy_schedule(1e-3, 5).abc
    # split factor capped at 2 here and in the single calls below: the
    # automatic factor depends on the call's tile count, and both sides must
    # sum in the same order
    plan = pe.Plan(Gs, T=5, abc=abc4, compute="bf16", force_class=3, tile=2, out_dtype=torch.float32,
                   ws_fill=0x5A, split_k=2)
    plan.launch(graph=False)
    torch.cuda.synchronize()
    cls, feats, _, flags = plan.selection()
    assert cls.tolist() == [3, 3, 3] and flags.tolist() == [0, 0, 0]
    T3, abc3 = class_schedule(pe, 3, abc4)
    for k, v in enumerate(vals):
        Y = pe.polar(Gs[k], T=T3, abc=abc3, compute="bf16", tile=2, out_dtype=torch.float32, split_k=2)
        torch.cuda.synchronize()
        assert relf(to_np(plan.outs[k]), to_np(Y)) <= 1e-6
        s_hat = np.linalg.svd(v / (1.01 * np.linalg.norm(v) + 1e-7), compute_uv=False)
        f_ref = OM.features(min(v.shape), max(v.shape), OM.moments_from_spectrum(s_hat))
        err = np.abs(feats[k] - f_ref).max()
        print(f"[learned] tile 256 case {k}: max feature err {err:.2e}", flush=True)
        assert err <= 2e-2
    plan.close()


@pytest.mark.parametrize("tile,m,n", [(1, 384, 640), (2, 512, 768)])
def test_combine_equals_a2_epilogue_bit_for_bit(pe, tile, m, n):
    """B = bA + cA^2 formed two ways gives the same bits: the learned path's
    combine kernel reads A row by row, the A^2 epilogue of the plain path reads
    A at the mirrored position (four rows of a column as one contiguous load).
    Equal outputs show that the stored A, diagonal tiles included, is exactly
    symmetric, which the mirrored read relies on."""
    import torch
    G, _ = _materialise(50 + tile, m, n, synth.spectrum_powerlaw(m, 1.0))
    abc4 = OS.greedy_schedule(1e-3, 5).abc
    plan = pe.Plan([G], T=5, abc=abc4, compute="bf16", force_class=2, tile=tile, out_dtype=torch.float32)
    plan.launch(graph=False)
    torch.cuda.synchronize()
    cls, _, _, flags = plan.selection()
    assert cls.tolist() == [2] and flags.tolist() == [0]
    T2, abc2 = class_schedule(pe, 2, abc4)
    Y = pe.polar(G, T=T2, abc=abc2, compute="bf16", tile=tile, out_dtype=torch.float32)
    torch.cuda.synchronize()
    diff = (plan.outs[0] - Y).abs().max().item()
    print(f"[learned] tile {tile} {m}x{n}: max |combine path - epilogue path| = {diff:.3e}", flush=True)
    assert torch.equal(plan.outs[0], Y)
    plan.close()


def test_learned_plan_with_fp8_steps(pe):
    """The learned path combined with e4m3 Gram-side steps on the 256 tile: the
    class is applied (forced), the result stays within the FP8 tolerance of the
    FP64 iteration with that class's schedule, and graph replays reproduce it."""
    import torch
    from tests.gpu_util import oracle_same_iteration
    G, v = _materialise(40, 768, 2304, synth.spectrum_powerlaw(768, 1.0))
    abc4 = OS.greedy_schedule(1e-3, 5).abc
    plan = pe.Plan([G], T=5, abc=abc4, compute="fp8", fp8_steps=3, force_class=2, tile=2,
                   out_dtype=torch.float32)
    plan.launch(graph=False)
    torch.cuda.synchronize()
    cls, _, _, _ = plan.selection()
    assert cls.tolist() == [2]
    ref = oracle_same_iteration(v, class_schedule(pe, 2, abc4)[1])
    err = relf(to_np(plan.outs[0]), ref)
    print(f"[learned] fp8 steps 3, class 2: relF {err:.3e}", flush=True)
    assert err <= 3e-2
    eager = plan.outs[0].clone()
    for _ in range(2):
        plan.launch(graph=True)
        torch.cuda.synchronize()
        assert torch.equal(plan.outs[0], eager)
    plan.close()


@pytest.mark.parametrize("fill", [0x00, 0x3F, 0xFF])
def test_learned_plan_ignores_workspace_contents(pe, fill):
    """The workspace needs no initialisation: whatever it held before (here
    every byte = fill, i.e. class slots reading 0, 0x3F3F3F3F or -1), a plan
    with a forced class gives the plain call's result with that class's
    schedule, eagerly and on graph replays."""
    import torch
    G, _ = _materialise(20, 320, 640, synth.spectrum_powerlaw(320, 1.0))
    abc4 = OS.greedy_schedule(1e-3, 5).abc
    print(f"[learned] workspace fill 0x{fill:02x}", flush=True)
    plan = pe.Plan([G], T=5, abc=abc4, compute="bf16", force_class=2, out_dtype=torch.float32,
                   ws_fill=fill)
    T2, abc2 = class_schedule(pe, 2, abc4)
    ref = pe.polar(G, T=T2, abc=abc2, compute="bf16", out_dtype=torch.float32)
    plan.launch(graph=False)
    torch.cuda.synchronize()
    assert relf(to_np(plan.outs[0]), to_np(ref)) <= 1e-6
    cls, _, _, flags = plan.selection()
    assert cls.tolist() == [2] and flags.tolist() == [0]
    for _ in range(2):
        plan.launch(graph=True)
        torch.cuda.synchronize()
        assert relf(to_np(plan.outs[0]), to_np(ref)) <= 1e-6
    plan.close()


def test_fallback_fires_and_matches_fixed_schedule(pe):
    """Forcing a short schedule of large l (class 2: l = 3e-2, 3 steps) on a
    spectrum reaching 1e-5 leaves small singular values unconverged: the
    ||X X^T - I|| estimate exceeds the threshold and the matrix is recomputed
    with the fixed schedule; a well-conditioned matrix the class suits is kept."""
    import torch
    G1, v1 = _materialise(10, 384, 768, np.geomspace(1, 1e-5, 384))
    G2, v2 = _materialise(11, 384, 768, np.linspace(1.0, 0.5, 384))
    abc4 = OS.greedy_schedule(1e-3, 5).abc
    plan = pe.Plan([G1, G2], T=5, abc=abc4, compute="bf16", force_class=2, fallback_tau=0.5,
                   out_dtype=torch.float32, ws_fill=0x3F)
    plan.launch(graph=False)
    torch.cuda.synchronize()
    cls, feats, est, flags = plan.selection()
    print(f"[fallback] classes {cls} estimates {est} flags {flags}", flush=True)
    assert flags.tolist() == [1, 0] and cls.tolist() == [4, 2]
    fixed = pe.polar(G1, T=5, abc=abc4, compute="bf16", out_dtype=torch.float32)
    T2, abc2 = class_schedule(pe, 2, abc4)
    forced = pe.polar(G2, T=T2, abc=abc2, compute="bf16", out_dtype=torch.float32)
    torch.cuda.synchronize()
    assert torch.equal(plan.outs[0], fixed)
    assert relf(to_np(plan.outs[1]), to_np(forced)) <= 1e-6
    # the estimate is a lower bound of ||X X^T - I||_2 that has converged here
    X1 = to_np(plan.outs[0])
    # (the reported estimate belongs to the first pass, before the re-run)
    Xf = to_np(pe.polar(G1, T=T2, abc=abc2, compute="bf16", out_dtype=torch.float32))
    M = Xf @ Xf.T - np.eye(Xf.shape[0])
    true = SP.spec_norm(M)
    assert est[0] <= true * (1 + 1e-3) and est[0] >= 0.9 * true
    # graph replays reproduce the eager result
    for _ in range(2):
        plan.launch(graph=True)
        torch.cuda.synchronize()
        assert torch.equal(plan.outs[0], fixed)
    plan.close()
