"""pe_polar_noalloc: the allocation-free variant of pe_polar (workspace in the
library's static device array) gives the same bits as pe_polar on the same
input, on two calls in a row with the second smaller, and rejects a matrix
whose workspace exceeds the array."""
import numpy as np
import pytest

import synth
from tests.gpu_util import device_input, oracle_same_iteration, oracle_schedule, relf, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import paper_2505_16932_amd as pe
    pe.lib()
    return pe


@pytest.mark.parametrize("compute,dtype", [("bf16", "bfloat16"), ("f32", "float32")])
def test_noalloc_matches_pe_polar(pe, compute, dtype):
    import torch
    dt = getattr(torch, dtype)
    abc = oracle_schedule(5)
    # first call larger (several tiles, split-K), second smaller and tall
    for shape, seed in [((640, 1800), 21), ((300, 130), 22)]:
        G64 = synth.powerlaw(seed, *shape).G
        G, vals = device_input(G64, dt)
        ref_out = pe.polar(G, T=5, abc=abc, compute=compute, out_dtype=torch.float32)
        out = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
        pe.polar_noalloc(G, out, T=5, abc=abc, compute=compute)
        torch.cuda.synchronize()
        print(f"[noalloc] {compute} {shape} equal={torch.equal(out, ref_out)}", flush=True)
        assert torch.equal(out, ref_out)
        err = relf(to_np(out), oracle_same_iteration(vals, abc))
        assert err <= (1e-5 if compute == "f32" else 3e-2), err


def test_noalloc_rejects_oversize(pe):
    import torch
    G = torch.zeros((4096, 8192), dtype=torch.bfloat16, device="cuda")
    need = pe.workspace_size([(4096, 8192)])
    assert need > pe.NOALLOC_SCRATCH_BYTES
    with pytest.raises(pe.PEError) as ei:
        pe.polar_noalloc(G, torch.empty_like(G), T=5)
    assert ei.value.status == 4
    assert "static scratch" in str(ei.value)
