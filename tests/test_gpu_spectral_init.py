"""The spectrum-aware initialisation step (appendix on matrices with large
spectral gaps, k = 1) through the C ABI against the oracle's same
construction in FP64: power method on the step-1 Gram matrix from the fixed
sign vector, the interpolating cubic, then the schedule.  Inputs with one
outlying singular value (the step applies) and without (it is the identity).

Bar: the path's own (1e-5 FP32, 3e-2 bf16) plus 2e-6 kappa, kappa = z^2 / w^2:
w^2 = ||X||_F^2 - z^2 cancels, so the FP32 power method's relative error in z
(~16 steps x 6e-8 = 1e-6) becomes 2e-6 kappa in w^2 and, through a ~ 1/w, in
the init cubic's action on the tail of the spectrum."""
import numpy as np
import pytest

import synth
from oracle import iteration as OI
from oracle import spectral_init as SI
from tests.gpu_util import device_input, oracle_same_iteration, oracle_schedule, relf, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import paper_2505_16932_amd as pe
    pe.lib()
    return pe


def _kappa(vals):
    """z^2 / w^2 of the oracle's construction on these input values."""
    m, n = vals.shape
    X = OI.normalise(vals.T if m > n else vals)
    A = X @ X.T
    z = SI.power_lower_bound(A, 16)
    return z * z / max(np.trace(A) - z * z, 1e-300)


def _outlier(seed, m, n):
    r = synth.rng(seed)
    k = min(m, n)
    sig = np.r_[1.0, 0.03 / np.arange(2, k + 1)]
    return synth.usv(r, m, n, sig).G


@pytest.mark.parametrize("compute,dtype,bar", [("f32", "float32", 1e-5), ("bf16", "bfloat16", 3e-2)])
@pytest.mark.parametrize("shape", [(200, 600), (600, 200), (512, 1536)])
def test_spectral_init_matches_oracle(pe, compute, dtype, bar, shape):
    import torch
    G, vals = device_input(_outlier(1700 + shape[0], *shape), getattr(torch, dtype))
    abc = oracle_schedule(5)
    X = pe.polar(G, T=5, abc=abc, compute=compute, out_dtype=torch.float32, spectral_init=16)
    torch.cuda.synchronize()
    ref = SI.spectrum_aware_polar_express(vals, abc, iters=16)
    e = relf(to_np(X), ref)
    kappa = _kappa(vals)
    print(f"[init] {compute} {shape} relF={e:.3e} kappa={kappa:.1f} bar={bar + 2e-6 * kappa:.2e}", flush=True)
    assert e <= bar + 2e-6 * kappa
    # the step made a difference: the plain iteration is far from it
    assert relf(oracle_same_iteration(vals, abc), ref) > 10 * bar


def test_spectral_init_identity_without_outlier(pe):
    """Gaussian input: z <= w, the init step is the identity, so the result is
    the ordinary iteration run for the same T (one extra Gram pass)."""
    import torch
    G, vals = device_input(synth.rng(1720).standard_normal((300, 900)), torch.float32)
    abc = oracle_schedule(5)
    X = pe.polar(G, T=5, abc=abc, compute="f32", out_dtype=torch.float32, spectral_init=8)
    torch.cuda.synchronize()
    assert relf(to_np(X), oracle_same_iteration(vals, abc)) <= 1e-5


def test_spectral_init_batched_mixed(pe):
    import torch
    shapes = [(256, 768), (384, 384), (700, 300)]
    Gs, vals = [], []
    for k, sh in enumerate(shapes):
        G64 = _outlier(1730 + k, *sh) if k != 1 else synth.rng(1731).standard_normal(sh)
        g, v = device_input(G64, torch.bfloat16)
        Gs.append(g)
        vals.append(v)
    abc = oracle_schedule(5)
    plan = pe.Plan(Gs, T=5, abc=abc, compute="bf16", out_dtype=torch.float32, spectral_init=16)
    plan.launch(graph=True)
    torch.cuda.synchronize()
    for X, v in zip(plan.outs, vals):
        assert relf(to_np(X), SI.spectrum_aware_polar_express(v, abc, iters=16)) <= 3e-2 + 2e-6 * _kappa(v)
    plan.close()
