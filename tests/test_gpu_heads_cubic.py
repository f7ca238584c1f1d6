"""Per-head splitting and the degree-3 schedule (Appendix G, application to
Muon; Appendix E, eq. deg3_solution), through the C ABI against the FP64
oracle on the same values.

* A QKV-shaped gradient (768 x 2304) split into 36 head blocks of 768 x 64 and
  an output projection (768 x 768) split by rows into 12 blocks of 64 x 768:
  one grouped call over the strided views, outputs written into the head
  blocks of full-size outputs (strided stores), every block against the oracle.
* The degree-3 schedule (c_t = 0: no A^2 product) in FP32 and bf16, single and
  batched, against the oracle's same iteration with the oracle's own cubic
  schedule."""
import numpy as np
import pytest

import synth
from oracle import schedule as OS
from tests.gpu_util import device_input, oracle_same_iteration, oracle_schedule, relf, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import paper_2505_16932_amd as pe
    pe.lib()
    return pe


def test_per_head_split_batched(pe):
    import torch
    qkv, qv = device_input(synth.powerlaw(1601, 768, 2304).G, torch.bfloat16)
    wo, wv = device_input(synth.powerlaw(1602, 768, 768).G, torch.bfloat16)
    heads = pe.split_heads(qkv, 36, axis=1) + pe.split_heads(wo, 12, axis=0)
    out_qkv = torch.zeros((768, 2304), dtype=torch.float32, device="cuda")
    out_wo = torch.zeros((768, 768), dtype=torch.float32, device="cuda")
    outs = pe.split_heads(out_qkv, 36, axis=1) + pe.split_heads(out_wo, 12, axis=0)
    abc = oracle_schedule(5)
    pe.polar_batched(heads, T=5, abc=abc, compute="bf16", outs=outs)
    torch.cuda.synchronize()
    worst = 0.0
    for h in range(36):
        ref = oracle_same_iteration(qv[:, 64 * h:64 * (h + 1)], abc)
        worst = max(worst, relf(to_np(out_qkv[:, 64 * h:64 * (h + 1)]), ref))
    for h in range(12):
        ref = oracle_same_iteration(wv[64 * h:64 * (h + 1), :], abc)
        worst = max(worst, relf(to_np(out_wo[64 * h:64 * (h + 1), :]), ref))
    print(f"[heads] 48 head blocks, worst relF {worst:.3e}", flush=True)
    assert worst <= 3e-2


@pytest.mark.parametrize("compute,dtype,bar", [("f32", "float32", 1e-5), ("bf16", "bfloat16", 3e-2)])
def test_cubic_schedule(pe, compute, dtype, bar):
    import torch
    T = 8
    c = pe.coeffs_cubic(1e-3, T)
    o = OS.greedy_schedule_cubic(1e-3, T).abc
    assert np.allclose(c.abc, o, rtol=1e-13)
    shapes = [(300, 900), (900, 300), (256, 256)]
    Gs, vals = [], []
    for k, sh in enumerate(shapes):
        g, v = device_input(synth.rng(1610 + k).standard_normal(sh), getattr(torch, dtype))
        Gs.append(g)
        vals.append(v)
    Xs = pe.polar_batched(Gs, T=T, abc=c.abc, compute=compute, out_dtype=torch.float32)
    X1 = pe.polar(Gs[0], T=T, abc=c.abc, compute=compute, out_dtype=torch.float32)
    torch.cuda.synchronize()
    for X, v, sh in zip(Xs, vals, shapes):
        e = relf(to_np(X), oracle_same_iteration(v, o))
        print(f"[cubic] {compute} {sh} T={T} relF={e:.3e}", flush=True)
        assert e <= bar
    assert relf(to_np(X1), to_np(Xs[0])) <= (1e-6 if compute == "f32" else 1e-2)
