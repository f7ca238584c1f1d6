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


def test_bf16_single_step(pe):
    """T = 1 on the bf16 path: the one update is also the last, so it reads the
    FP32 master of X_0 (the bf16 copy stands in for X_0 only from T = 2)."""
    import torch
    G, v = device_input(synth.powerlaw(951, 300, 520).G, torch.bfloat16)
    abc = OS.greedy_schedule(1e-3, 1).abc
    X = pe.polar(G, T=1, abc=abc, compute="bf16", out_dtype=torch.float32)
    torch.cuda.synchronize()
    e = relf(to_np(X), oracle_same_iteration(v, abc))
    print(f"[edge] bf16 T=1 relF={e:.3e}", flush=True)
    assert e <= 3e-2


def test_bf16_call_mixing_input_types(pe):
    """bf16 and FP32 inputs in one bf16 call: X_0 of the FP32 input is not
    exactly its bf16 copy, so the whole call keeps the FP32 master of X_0."""
    import torch
    abc = OS.greedy_schedule(1e-3, 5).abc
    g0, v0 = device_input(synth.rng(952).standard_normal((260, 700)), torch.bfloat16)
    g1, v1 = device_input(synth.rng(953).standard_normal((700, 260)), torch.float32)
    Xs = pe.polar_batched([g0, g1], T=5, abc=abc, compute="bf16", out_dtype=torch.float32)
    torch.cuda.synchronize()
    for X, v in zip(Xs, (v0, v1)):
        e = relf(to_np(X), oracle_same_iteration(v, abc))
        print(f"[edge] mixed-input bf16 call {v.shape} relF={e:.3e}", flush=True)
        assert e <= 3e-2


@pytest.mark.parametrize("compute,dtype", [("f32", "float32"), ("bf16", "bfloat16")])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_input_gives_nan_output(pe, compute, dtype, bad):
    """A NaN or infinite entry makes ||G||_F, and with it the scale of X_0, NaN
    or zero-times-infinity: every entry of the result is NaN.  The library
    reports no status for it (the call is asynchronous); the other matrices of
    a batched call are unaffected."""
    import torch
    abc = OS.greedy_schedule(1e-3, 5).abc
    g_bad, _ = device_input(synth.rng(954).standard_normal((200, 300)), getattr(torch, dtype))
    g_bad[17, 123] = bad
    g_ok, v_ok = device_input(synth.rng(955).standard_normal((200, 300)), getattr(torch, dtype))
    X_bad, X_ok = pe.polar_batched([g_bad, g_ok], T=5, abc=abc, compute=compute, out_dtype=torch.float32)
    torch.cuda.synchronize()
    assert torch.isnan(X_bad).all().item()
    tol = 1e-5 if compute == "f32" else 3e-2
    assert relf(to_np(X_ok), oracle_same_iteration(v_ok, abc)) <= tol
