"""The fused Muon step (Section 1.1) through the C ABI against the oracle's
step in FP64 on the same values: the momentum update in the norm pass, the
weight step in the last update's epilogue, the iteration running on the new
momentum.  FP32 compute: the momentum to FP32 rounding and the step direction
(W - W') / lr within 1e-5; bf16: the direction within 3e-2 and bf16 weights
within a few bf16 ulps of the oracle's."""
import numpy as np
import pytest

import synth
from oracle import muon as MU
from tests.gpu_util import device_input, oracle_schedule, relf, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pe():
    import paper_2505_16932_amd as pe
    pe.lib()
    return pe


def _state(shape, seed, torch, wdtype):
    r = synth.rng(seed)
    G, gvals = device_input(synth.powerlaw(seed, *shape).G * 3.0, torch.bfloat16)
    M = torch.from_numpy((0.02 * r.standard_normal(shape)).astype(np.float32)).cuda()
    W = torch.from_numpy(r.standard_normal(shape).astype(np.float32)).to(wdtype).cuda()
    return G, gvals, M, W


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_muon_step_matches_oracle(pe, compute):
    import torch
    shapes = [(300, 700), (700, 300), (768, 2304)]
    lr, beta, wd = (1.0, 0.9, 0.0) if compute == "f32" else (1.0, 0.95, 0.1)
    abc = oracle_schedule(5)
    Gs, gv, Ms, Ws = [], [], [], []
    for k, sh in enumerate(shapes):
        G, g, M, W = _state(sh, 1500 + k, torch, torch.float32)
        Gs.append(G); gv.append(g); Ms.append(M); Ws.append(W)
    M0 = [to_np(M) for M in Ms]
    W0 = [to_np(W) for W in Ws]
    outs = pe.muon_step(Gs, Ms, Ws, lr=lr, beta=beta, wd=wd, T=5, abc=abc, compute=compute)
    torch.cuda.synchronize()
    assert all(o is None for o in outs)
    bar = 1e-5 if compute == "f32" else 3e-2
    for k in range(len(shapes)):
        Mr, Xr, Wr = MU.muon_step(gv[k], M0[k], W0[k], abc, lr=lr, beta=beta, wd=wd)
        em = relf(to_np(Ms[k]), Mr)
        direction = ((1 - lr * wd) * W0[k] - to_np(Ws[k])) / lr
        ex = relf(direction, Xr)
        print(f"[muon] {compute} {shapes[k]} momentum relF={em:.2e} direction relF={ex:.3e}", flush=True)
        assert em <= 1e-6
        assert ex <= bar


def test_muon_bf16_weights_and_output(pe):
    """bf16 weights updated in place; the output X is written as well when given."""
    import torch
    abc = oracle_schedule(5)
    G, g, M, W = _state((512, 1024), 1510, torch, torch.bfloat16)
    M0, W0 = to_np(M), to_np(W)
    X = torch.empty((512, 1024), dtype=torch.float32, device="cuda")
    pe.muon_step([G], [M], [W], lr=0.02, beta=0.9, T=5, abc=abc, compute="bf16", outs=[X])
    torch.cuda.synchronize()
    Mr, Xr, Wr = MU.muon_step(g, M0, W0, abc, lr=0.02, beta=0.9)
    assert relf(to_np(X), Xr) <= 3e-2
    # W' = bf16(W - lr X): within a bf16 rounding of the oracle's W' plus lr |dX|
    d = np.abs(to_np(W) - Wr)
    assert np.all(d <= 2.0 ** -8 * np.abs(Wr) + 0.02 * 0.05 + 1e-6)


@pytest.mark.parametrize("wdtype,with_out", [("bf16", True), ("bf16", False), ("f32", False), ("f32", True)])
def test_muon_large_tile_staged_weight_step(pe, wdtype, with_out):
    """The 256 tile's last update stages X_T in LDS and applies the weight step
    by whole rows (16-byte accesses, ragged edges element by element, a
    transposed matrix in the caller's layout): the momentum and the step
    against the oracle; with a bf16 output and no decay, W' is
    W - lr X_out rounded once, X_out being the output's own bf16 values."""
    import torch
    abc = oracle_schedule(5)
    shapes = [(300, 700), (700, 300), (512, 1024)]
    wt = torch.bfloat16 if wdtype == "bf16" else torch.float32
    lr, beta, wd = (0.02, 0.9, 0.0) if with_out else (0.02, 0.95, 0.1)
    Gs, gv, Ms, Ws = [], [], [], []
    for k, sh in enumerate(shapes):
        G, g, M, W = _state(sh, 1560 + k, torch, wt)
        Gs.append(G); gv.append(g); Ms.append(M); Ws.append(W)
    M0 = [to_np(M) for M in Ms]
    W0 = [to_np(W) for W in Ws]
    outs = [torch.empty(sh, dtype=torch.bfloat16, device="cuda") for sh in shapes] if with_out else None
    pe.muon_step(Gs, Ms, Ws, lr=lr, beta=beta, wd=wd, T=5, abc=abc, compute="bf16", outs=outs, tile=2)
    torch.cuda.synchronize()
    for k, sh in enumerate(shapes):
        Mr, Xr, Wr = MU.muon_step(gv[k], M0[k], W0[k], abc, lr=lr, beta=beta, wd=wd)
        assert relf(to_np(Ms[k]), Mr) <= 1e-6
        Wk = to_np(Ws[k])
        if wdtype == "f32":
            ex = relf(((1 - lr * wd) * W0[k] - Wk) / lr, Xr)
            print(f"[muon] 256 tile {sh} f32 W: direction relF={ex:.3e}", flush=True)
            assert ex <= 3e-2
        else:
            d = np.abs(Wk - Wr)
            assert np.all(d <= 2.0 ** -8 * np.abs(Wr) + lr * 0.05 + 1e-6)
        if with_out:
            Xo = to_np(outs[k])
            assert relf(Xo, Xr) <= 3e-2
            # one FP32 fused multiply-add, then the weight's own rounding
            w32 = (W0[k] - float(np.float32(lr)) * Xo).astype(np.float32)
            Wexp = torch.from_numpy(w32).to(wt).to(torch.float64).numpy()
            bad = int(np.count_nonzero(Wk != Wexp))
            print(f"[muon] 256 tile {sh} {wdtype} W with bf16 output: {bad} weights differ", flush=True)
            assert bad == 0


@pytest.mark.parametrize("wdtype", ["bf16", "f32"])
def test_muon_large_tile_strided_weights(pe, wdtype):
    """Weights, momentum and output as column views of wider arrays (row pitch
    1024 or 512 elements, 700 or 300 columns): the staged weight step takes its
    16-byte path up to the last whole chunk of a row and the element path for
    the ragged rest, and leaves the columns past the view untouched."""
    import torch
    abc = oracle_schedule(5)
    wt = torch.bfloat16 if wdtype == "bf16" else torch.float32
    shapes, pitches = [(300, 700), (700, 300)], [1024, 512]
    lr = 0.02
    Gs, Ms, Ws, Wbig, outs = [], [], [], [], []
    W0, Wbig0 = [], []
    for k, (sh, pitch) in enumerate(zip(shapes, pitches)):
        G, g, M, W = _state(sh, 1580 + k, torch, wt)
        big = torch.from_numpy(synth.rng(1590 + k).standard_normal((sh[0], pitch)).astype(np.float32)).to(wt).cuda()
        big[:, :sh[1]] = W
        Mbig = torch.zeros((sh[0], pitch), dtype=torch.float32, device="cuda")
        Mbig[:, :sh[1]] = M
        Obig = torch.zeros((sh[0], pitch), dtype=torch.bfloat16, device="cuda")
        Gs.append(G); Ms.append(Mbig[:, :sh[1]]); Ws.append(big[:, :sh[1]]); Wbig.append(big)
        outs.append(Obig[:, :sh[1]])
        W0.append(to_np(W)); Wbig0.append(to_np(big))
    pe.muon_step(Gs, Ms, Ws, lr=lr, beta=0.9, wd=0.0, T=5, abc=abc, compute="bf16", outs=outs, tile=2)
    torch.cuda.synchronize()
    for k, sh in enumerate(shapes):
        Xo = to_np(outs[k])
        w32 = (W0[k] - float(np.float32(lr)) * Xo).astype(np.float32)
        Wexp = torch.from_numpy(w32).to(wt).to(torch.float64).numpy()
        Wk = to_np(Wbig[k])
        bad = int(np.count_nonzero(Wk[:, :sh[1]] != Wexp))
        print(f"[muon] strided {wdtype} W {sh} pitch {pitches[k]}: {bad} weights differ", flush=True)
        assert bad == 0
        assert np.array_equal(Wk[:, sh[1]:], Wbig0[k][:, sh[1]:])


def test_muon_plan_replays_are_successive_steps(pe):
    """A plan captured with the Muon fields applies one step per launch: two
    launches equal two oracle steps with the same gradient."""
    import torch
    abc = oracle_schedule(5)
    G, g, M, W = _state((256, 640), 1520, torch, torch.float32)
    M0, W0 = to_np(M), to_np(W)
    plan = pe.Plan([G], outs=[None], T=5, abc=abc, compute="f32", moms=[M], weights=[W],
                   muon=(0.9, 1.0, 0.0))
    plan.launch(graph=True)
    plan.launch(graph=True)
    torch.cuda.synchronize()
    M1, _, W1 = MU.muon_step(g, M0, W0, abc, lr=1.0, beta=0.9)
    M2, X2, W2 = MU.muon_step(g, M1, W1, abc, lr=1.0, beta=0.9)
    assert relf(to_np(M), M2) <= 1e-6
    assert relf(W1 - to_np(W), X2) <= 1e-5
    plan.close()


def test_muon_rejects_fallback_combination(pe):
    import torch
    G = torch.ones((64, 128), dtype=torch.bfloat16, device="cuda")
    M = torch.zeros((64, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(pe.PEError) as ei:
        pe.polar_batched([G], T=5, moms=[M], muon=(0.9, 0.1, 0.0), force_class=4, fallback_tau=0.1)
    assert ei.value.status == 2


def test_muon_with_fast_iteration(pe):
    """The Muon step on the fast rectangular iteration (FP32, restart 3, no
    shift): momentum in the norm pass, polar(M) by Algorithm 4, the weight step
    in the fast path's final update; against the oracle's momentum, its
    Algorithm 4 on that momentum and the weight step (bar 2e-4, the fast
    path's own)."""
    import torch
    from oracle import fastapply as FA
    abc = oracle_schedule(5)
    G, g, M, W = _state((300, 1100), 1530, torch, torch.float32)
    M0, W0 = to_np(M), to_np(W)
    lr, beta, wd = 0.5, 0.9, 0.1
    pe.muon_step([G], [M], [W], lr=lr, beta=beta, wd=wd, T=5, abc=abc, compute="f32",
                 fast_restart=3, fast_eps=0.0)
    torch.cuda.synchronize()
    Mr = beta * M0 + (1.0 - beta) * g
    Xr = FA.fast_polar_express(Mr, abc, restart=3, eps=0.0)
    direction = ((1 - lr * wd) * W0 - to_np(W)) / lr
    em, ex = relf(to_np(M), Mr), relf(direction, Xr)
    print(f"[muon] fast iteration: momentum relF={em:.2e} direction relF={ex:.3e}", flush=True)
    assert em <= 1e-6 and ex <= 2e-4


@pytest.mark.parametrize("compute,bar", [("f32", 1e-5), ("bf16", 3e-2)])
def test_muon_with_spectral_init(pe, compute, bar):
    """The Muon step with the spectrum-aware initialisation (16 power steps)
    on a momentum with one outlying singular value; against the oracle's
    momentum, its initialised iteration on that momentum and the weight step
    (bar: the path's own plus 2e-6 kappa, as for the initialisation alone)."""
    import torch
    from oracle import iteration as OI
    from oracle import spectral_init as SI
    abc = oracle_schedule(5)
    r = synth.rng(1540)
    m, n = 256, 768
    sig = np.r_[1.0, 0.03 / np.arange(2, m + 1)]
    G, g = device_input(synth.usv(r, m, n, sig).G, torch.bfloat16)
    M = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    W = torch.from_numpy(r.standard_normal((m, n)).astype(np.float32)).cuda()
    W0 = to_np(W)
    lr, beta = 1.0, 0.5
    pe.muon_step([G], [M], [W], lr=lr, beta=beta, T=5, abc=abc, compute=compute, spectral_init=16)
    torch.cuda.synchronize()
    Mr = (1.0 - beta) * g
    Xr = SI.spectrum_aware_polar_express(Mr, abc, iters=16)
    X0 = OI.normalise(Mr)
    A = X0 @ X0.T
    z = SI.power_lower_bound(A, 16)
    kappa = z * z / max(np.trace(A) - z * z, 1e-300)
    ex = relf(W0 - to_np(W), Xr)
    print(f"[muon] spectral init {compute}: direction relF={ex:.3e} kappa={kappa:.1f}", flush=True)
    assert relf(to_np(M), Mr) <= 1e-6
    assert ex <= bar + 2e-6 * kappa
