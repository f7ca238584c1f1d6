"""Edge cases of the boundary through the C ABI against the FP64 oracle:
degenerate shapes (a 1 x 1 matrix, row and column vectors, 2 x 2, a 3 x 17
whose smaller side is below 16 and so runs with FP32 operands on every path)
and the limits of the step count (T = 1 and the maximum T = 64, where the
schedule repeats its Newton-Schulz step).  Bar: 1e-5 (FP32 arithmetic)."""
import numpy as np
import pytest

import synth
from oracle import schedule as OS
from tests.gpu_util import device_input, oracle_same_iteration, relf, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import paper_2505_16932_amd as pe
    pe.lib()
    return pe


@pytest.mark.parametrize("compute,dtype", [("f32", "float32"), ("bf16", "bfloat16")])
def test_degenerate_shapes(pe, compute, dtype):
    import torch
    shapes = [(1, 1), (1, 7), (7, 1), (1, 1000), (1000, 1), (2, 2), (3, 17)]
    abc = OS.greedy_schedule(1e-3, 5).abc
    Gs, vals = [], []
    for k, sh in enumerate(shapes):
        g, v = device_input(synth.rng(900 + k).standard_normal(sh), getattr(torch, dtype))
        Gs.append(g)
        vals.append(v)
    Xs = pe.polar_batched(Gs, T=5, abc=abc, compute=compute, out_dtype=torch.float32)
    torch.cuda.synchronize()
    for X, v, sh in zip(Xs, vals, shapes):
        ref = oracle_same_iteration(v, abc)
        e = relf(to_np(X), ref)
        print(f"[edge] {compute} {sh} relF={e:.3e}", flush=True)
        assert X.shape == sh and e <= 1e-5
    # a single matrix through the one-matrix entry point as well
    X = pe.polar(Gs[0], T=5, abc=abc, compute=compute, out_dtype=torch.float32)
    torch.cuda.synchronize()
    assert relf(to_np(X), oracle_same_iteration(vals[0], abc)) <= 1e-5


@pytest.mark.parametrize("T", [1, 64])
def test_step_count_limits(pe, T):
    import torch
    G, v = device_input(synth.powerlaw(950, 300, 520).G, torch.float32)
    abc = OS.greedy_schedule(1e-3, T).abc
    X = pe.polar(G, T=T, abc=abc, compute="f32", out_dtype=torch.float32)
    torch.cuda.synchronize()
    e = relf(to_np(X), oracle_same_iteration(v, abc))
    print(f"[edge] T={T} relF={e:.3e}", flush=True)
    assert e <= 1e-5


def test_step_count_out_of_range_rejected(pe):
    import torch
    G = torch.ones((16, 16), device="cuda")
    abc = np.tile(OS.greedy_schedule(1e-3, 8).abc[-1], (65, 1))
    with pytest.raises(Exception):
        pe.polar(G, T=65, abc=abc, compute="f32")
