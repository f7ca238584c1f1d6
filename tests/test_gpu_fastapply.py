"""The fast rectangular iteration (Appendix G, Algorithm 4; FP32 compute)
through the C ABI against the oracle's Algorithm 4 in FP64 on the same input
values: restart intervals 1-3, with and without the first segment's shift,
wide and tall, ragged tiles, for the whole matrix and every 256 x 256 block.

Bar 2e-4, derived from the arithmetic: a segment ends with X <- q X + D X where
q = prod a_t (up to 8.2 * 4.07 * 3.91 = 130 over three steps of the l = 1e-3
schedule) and D X nearly cancels q X on the large singular values, so the
FP32 rounding of the products (6e-8 relative, about 25 products deep) is
scaled by q: 130 * 6e-8 * 25 = 2e-4.  (The ordinary FP32 path's 1e-5 bar
stays for the ordinary path.)  Longer segments grow q to 976 (five steps)
and lose FP32 accuracy altogether (4e-2 measured); they are not offered as a
parity case."""
import numpy as np
import pytest

import synth
from oracle import fastapply as FA
from tests.gpu_util import device_input, oracle_same_iteration, oracle_schedule, relf, tile_relf, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import paper_2505_16932_amd as pe
    pe.lib()
    return pe


def _input(kind, shape, seed):
    r = synth.rng(seed)
    s = min(shape)
    if kind == "gauss":
        return r.standard_normal(shape)
    if kind == "loguniform":
        return synth.usv(r, shape[0], shape[1], synth.spectrum_loguniform(r, s, 1e-2, 1.0)).G
    return synth.usv(r, shape[0], shape[1], synth.spectrum_powerlaw(s)).G


BAR = 2e-4
CASES = [("gauss", (300, 1100), 3, 1e-3), ("gauss", (1100, 300), 2, 0.0), ("loguniform", (260, 900), 3, 0.0),
         ("loguniform", (260, 900), 1, 1e-3), ("powerlaw", (384, 1400), 2, 1e-3), ("gauss", (130, 130), 3, 1e-3),
         ("loguniform", (128, 2048), 3, 0.0)]


@pytest.mark.parametrize("kind,shape,restart,eps", CASES)
def test_fast_iteration_matches_oracle(pe, kind, shape, restart, eps):
    import torch
    G64 = _input(kind, shape, 800 + shape[0] + restart)
    G, vals = device_input(G64, torch.float32)
    abc = oracle_schedule(5)
    X = pe.polar(G, T=5, abc=abc, compute="f32", out_dtype=torch.float32, fast_restart=restart,
                 fast_eps=eps)
    torch.cuda.synchronize()
    ref = FA.fast_polar_express(vals, abc, restart=restart, eps=eps)
    Xn = to_np(X)
    e, t = relf(Xn, ref), tile_relf(Xn, ref)
    print(f"[fast] {kind} {shape} restart={restart} eps={eps} relF={e:.3e} max-block={t:.3e}", flush=True)
    assert e <= BAR and t <= BAR


def test_unshifted_fast_iteration_equals_ordinary_path(pe):
    """eps = 0: the same composite as the ordinary iteration (to the bar above)."""
    import torch
    G64 = _input("loguniform", (256, 1000), 850)
    G, vals = device_input(G64, torch.float32)
    abc = oracle_schedule(5)
    X1 = pe.polar(G, T=5, abc=abc, compute="f32", out_dtype=torch.float32, fast_restart=3, fast_eps=0.0)
    X0 = pe.polar(G, T=5, abc=abc, compute="f32", out_dtype=torch.float32)
    torch.cuda.synchronize()
    assert relf(to_np(X1), to_np(X0)) <= BAR
    assert relf(to_np(X1), oracle_same_iteration(vals, abc)) <= BAR


def test_fast_iteration_batched_and_graph(pe):
    import torch
    shapes = [(256, 768), (768, 256), (200, 650)]
    Gs, vals = [], []
    for k, sh in enumerate(shapes):
        g, v = device_input(_input("gauss", sh, 860 + k), torch.float32)
        Gs.append(g)
        vals.append(v)
    abc = oracle_schedule(5)
    plan = pe.Plan(Gs, T=5, abc=abc, compute="f32", fast_restart=3, fast_eps=1e-3)
    eager = [x.clone() for x in plan.launch(graph=False)]
    for _ in range(3):
        plan.launch(graph=True)
        torch.cuda.synchronize()
        for a, b in zip(plan.outs, eager):
            assert torch.equal(a, b)
    for X, v in zip(plan.outs, vals):
        assert relf(to_np(X), FA.fast_polar_express(v, abc, 3, 1e-3)) <= BAR
    plan.close()


def test_fast_iteration_rejects_bf16(pe):
    import torch
    G = torch.ones((64, 256), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(pe.PEError) as ei:
        pe.polar(G, T=5, compute="bf16", fast_restart=3)
    assert ei.value.status == 2
