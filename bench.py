#!/usr/bin/env python3
"""Polar Express throughput on one MI355X.

One step = one pass of the whole method (norm + T polynomial steps) over every
matrix of the workload, through a plan (grouped launches captured as a
hipGraph).  Inputs are synthetic, seeded, resident in HBM before timing.

Workloads:
  wide-batch        32-layer 4096-wide model: per layer four 4096x4096 and three
                    4096x14336 bf16 matrices (224), sigma_i = 1/i, Haar singular
                    vectors, T = 5, bf16 MFMA operands with FP32 accumulation
                    and FP32 master iterate (default); the e4m3 variant (Gram-side
                    products of steps 1-3 in e4m3) is timed after it and reported
                    under "fp8_variant"
  wide-layer        one layer of the above (7 matrices), for profiler runs
  gpt-small-batch   12 layers x {768x2304, 768x768, 768x3072, 3072x768} (48), sigma_i = 1/i
  single-4096x1024  one 4096x1024 bf16 matrix, log-uniform spectrum
  small-256         one 256x256 FP32 matrix, iid N(0,1) (latency-bound: read ms_per_step)

Metric: algorithmic TFLOP/s = sum over matrices and steps of (3 s^2 L + s^3)
(s = min(m,n), L = max(m,n): Gram s^2 L, A^2 s^3 on the symmetric half, B X
2 s^2 L) divided by the wall time of the step.  pct_mfma_peak weights each
product by the dense peak of its precision (bf16 2.5, e4m3 5.0 PFLOP/s).
dense_equivalent_tflops counts the products as plain GEMMs instead
(4 s^2 L + 2 s^3: full Gram and A^2, the paper's multiply-add count x 2).
The comparison path runs the same matrices one plain bf16 call at a time.
Accuracy: ||X_T - U V^T||_2 for every matrix (U V^T known by construction;
power iteration on the device), its prediction from the scalar composite on
the known spectrum (max_i |1 - phi_T(sigma_i / (1.01 ||G||_F))|), and the
relative Frobenius distance of the GPU result from the FP64 oracle's same
iteration on the matrix the CPU baseline runs.
fast_rect_f32 (wide workloads): the rectangular fast iteration (restart every
3 steps) against the standard iteration, both FP32, on three 4096x14336
matrices: ms per call and the polar error of each result.
muon_step, spectral_init, per_head (wide workloads, bf16): the fused Muon
optimizer step over all matrices, the spectrum-aware initialisation, and the
first layer's 4096x4096 matrices split into 32 heads of 4096x128, each timed
against the corresponding plain plan.

Prints ONE JSON line (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algo_flops(shapes, T):
    tot = 0.0
    for m, n in shapes:
        s, L = min(m, n), max(m, n)
        tot += 3.0 * s * s * L + float(s) ** 3
    return tot * T


def dense_flops(shapes, T):
    tot = 0.0
    for m, n in shapes:
        s, L = min(m, n), max(m, n)
        tot += 4.0 * s * s * L + 2.0 * float(s) ** 3
    return tot * T


def update_flops(shapes):
    return sum(2.0 * min(m, n) ** 2 * max(m, n) for m, n in shapes)


def make_workload(name, torch, device, inputs="spectral"):
    import synth
    if inputs == "gaussian":
        # iid N(0,1) entries of the same shapes: no QR, for profiler runs only
        # (kernel time does not depend on the spectrum)
        shapes = {"wide-batch": synth.WIDE_LAYER_SHAPES * 32, "wide-layer": synth.WIDE_LAYER_SHAPES,
                  "gpt-small-batch": synth.GPT_SMALL_SHAPES * 12, "single-4096x1024": [(4096, 1024)]}[name]
        g = torch.Generator(device=device)
        g.manual_seed(7)
        Gs = [torch.randn(s, generator=g, device=device, dtype=torch.float32).to(torch.bfloat16)
              for s in shapes]
        return Gs, 5, dict(gaussian=True)
    if name == "wide-batch":
        mats, templates = synth.torch_layer_batch(32, seed=1004, device=device)
        Gs = [m[0] for m in mats]
        meta = dict(mats=mats, templates=templates)
        return Gs, 5, meta
    if name == "wide-layer":
        mats, templates = synth.torch_layer_batch(1, seed=1004, device=device)
        return [m[0] for m in mats], 5, dict(mats=mats, templates=templates)
    if name == "gpt-small-batch":
        mats, templates = synth.torch_layer_batch(12, seed=1003, device=device,
                                                  shapes=synth.GPT_SMALL_SHAPES)
        return [m[0] for m in mats], 5, dict(mats=mats, templates=templates)
    if name == "small-256":
        import numpy as np
        G64 = synth.rng(1001).standard_normal((256, 256))
        U, _, Vt = np.linalg.svd(G64)   # reference polar factor, for the error printout only
        G = torch.from_numpy(G64.astype("float32")).to(device)
        return [G], 5, dict(polar=torch.from_numpy(U @ Vt).float().to(device))
    if name == "single-4096x1024":
        S = synth.loguniform(1002)
        G = torch.from_numpy(S.G.astype("float32")).to(torch.bfloat16).to(device)
        return [G], 5, dict(synth=S)
    raise SystemExit(f"unknown workload {name}")


def factors(meta, idx):
    """(U', V) with U' V^T the polar factor of matrix idx (known by construction)."""
    G, perm, signs, j = meta["mats"][idx]
    U, sig, V = meta["templates"][j]
    return U[:, perm] * signs, V


def polar_factor(meta, idx, torch):
    """U' V^T of matrix idx (known by construction)."""
    if "polar" in meta:
        return meta["polar"]
    if "mats" in meta:
        Up, V = factors(meta, idx)
        return Up @ V.T
    S = meta["synth"]
    return torch.from_numpy(S.polar()).float().cuda()


def spec_norm_gpu(D, torch, iters=60):
    """||D||_2 by power iteration on D^T D (measurement only)."""
    g = torch.Generator(device=D.device)
    g.manual_seed(0)
    v = torch.randn(D.shape[1], 1, device=D.device, generator=g, dtype=torch.float32)
    v /= v.norm()
    lam = torch.zeros((), device=D.device)
    for _ in range(iters):
        w = D.T @ (D @ v)
        lam = w.norm()
        v = w / lam
    return float(lam.sqrt())


def spec_norm_factored(X, Up, V, torch, iters=40):
    """||X - Up V^T||_2 by power iteration, the difference applied through its
    factors (no m x n temporary; measurement only)."""
    X = X.float()
    g = torch.Generator(device=X.device)
    g.manual_seed(0)
    v = torch.randn(X.shape[1], device=X.device, generator=g, dtype=torch.float32)
    v /= v.norm()
    for _ in range(iters):
        y = X @ v - Up @ (V.T @ v)
        w = X.T @ y - V @ (Up.T @ y)
        v = w / w.norm()
    return float((X @ v - Up @ (V.T @ v)).norm())


def polar_errors(outs, meta, torch):
    """||X_T - U V^T||_2 of every matrix of the workload."""
    errs = []
    for idx, X in enumerate(outs):
        if "mats" in meta:
            Up, V = factors(meta, idx)
            errs.append(spec_norm_factored(X, Up, V, torch))
        else:
            errs.append(spec_norm_gpu(X.float() - polar_factor(meta, idx, torch).float(), torch))
    return errs


def predicted_polar_error(sigma, abc):
    """max_i |1 - phi_T(sigma_i / (1.01 ||G||_F + 1e-7))| for a known spectrum:
    the polar error of the exact iteration (the matrix error is the scalar
    composite's error on the normalised singular values)."""
    import numpy as np
    sigma = np.asarray(sigma, dtype=np.float64)
    x = sigma / (1.01 * np.sqrt(np.sum(sigma ** 2)) + 1e-7)
    for a, b, c in np.asarray(abc, dtype=np.float64).reshape(-1, 3):
        y = x * x
        x = x * (a + y * (b + c * y))
    return float(np.max(np.abs(1.0 - x)))


def err_summary(errs):
    import numpy as np
    e = np.asarray(errs)
    return dict(min=round(float(e.min()), 5), max=round(float(e.max()), 5),
                mean=round(float(e.mean()), 5))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_plan(plan, steps, warmup, stream, torch):
    for _ in range(warmup):
        plan.launch(graph=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        plan.launch(graph=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    return ev0.elapsed_time(ev1) / steps, wall / steps * 1e3


def measured_traffic(workload, compute, tile, fp8_steps):
    """HBM bytes per update launch from the committed counter runs, when they were
    taken on this workload and on the kernel source as it is now (else None).  The
    update runs in bf16 whether or not the Gram-side products of early steps use e4m3."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload.replace('-', '_')}.json")
    if compute == "f32" or tile != 0 or not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
        src = os.path.join(ROOT, "paper_2505_16932_amd", "csrc", "kernels.hip")
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != t["kernels_hip_sha256"]:
                return None
        return dict(gb=round((t["fetch_bytes"] + t["write_bytes"]) / 1e9, 2),
                    read_gb=round(t["fetch_bytes"] / 1e9, 2), write_gb=round(t["write_bytes"] / 1e9, 2))
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(mats, abc, T):
    """The FP64 oracle on the host cores, on a bounded sample of the workload
    (the given matrices, about 10-30 s of host work for the wide batch).
    Returns the baseline record and the oracle's result for the last matrix."""
    from oracle import iteration as OI
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    t0 = time.perf_counter()
    ref = None
    for G in mats:
        ref = OI.polar_express(G, abc)
    dt = time.perf_counter() - t0
    shapes = [tuple(G.shape) for G in mats]
    fl = algo_flops(shapes, T)
    desc = ", ".join(f"{m}x{n}" for m, n in shapes)
    return dict(value=fl / dt / 1e12, unit="TFLOP/s", cores=int(cores), kind="oracle",
                cpu=cpu_model(),
                sample=f"{len(mats)} of the workload's matrices ({desc}), T={T}, FP64 NumPy, {dt:.1f} s"), ref


def fast_row(Gs, meta, abc, T, args, stream, torch, log):
    """The rectangular fast iteration (restart every 3 steps, no shift) against
    the standard iteration, both FP32, on the three 4096x14336 matrices of the
    first layer: ms per call and the polar error of every result."""
    import paper_2505_16932_amd as pe
    idx = [i for i, G in enumerate(Gs) if max(G.shape) >= 3 * min(G.shape)][:3]
    sub = [Gs[i] for i in idx]
    fl = algo_flops([tuple(G.shape) for G in sub], T)
    row = dict(matrices=len(sub), shape=list(sub[0].shape), T=T, compute="f32", restart=3, eps=0.0)
    for name, kw in (("standard", {}), ("fast", dict(fast_restart=3, fast_eps=0.0))):
        plan = pe.Plan(sub, T=T, abc=abc, compute="f32", **kw)
        ms, _ = time_plan(plan, max(2, min(args.steps, 5)), 1, stream, torch)
        plan.launch(graph=True)
        torch.cuda.synchronize()
        errs = [spec_norm_factored(plan.outs[k], *factors(meta, i), torch) for k, i in enumerate(idx)]
        row[name] = dict(ms_per_call=round(ms, 3), algorithmic_tflops=round(fl / (ms * 1e-3) / 1e12, 2),
                         polar_err=[round(e, 5) for e in errs])
        plan.close()
        del plan
        torch.cuda.empty_cache()
    row["speedup"] = round(row["standard"]["ms_per_call"] / row["fast"]["ms_per_call"], 3)
    log(f"[bench] fast rectangular iteration (FP32, {len(sub)} x {tuple(sub[0].shape)}): "
        f"{row['fast']['ms_per_call']} ms against {row['standard']['ms_per_call']} ms "
        f"(polar error {row['fast']['polar_err']} vs {row['standard']['polar_err']})")
    return row


def muon_row(Gs, abc, T, args, stream, torch, log, base_ms):
    """The fused Muon optimizer step over the whole workload (bf16 weights,
    FP32 momentum; no X output): ms per step against the plain plan's."""
    import paper_2505_16932_amd as pe
    moms = [torch.zeros(G.shape, dtype=torch.float32, device=G.device) for G in Gs]
    weights = [torch.zeros(G.shape, dtype=torch.bfloat16, device=G.device) for G in Gs]
    plan = pe.Plan(Gs, outs=[None] * len(Gs), T=T, abc=abc, compute="bf16", moms=moms, weights=weights,
                   muon=(0.95, 0.02, 0.01))
    ms, _ = time_plan(plan, max(2, min(args.steps, 5)), 1, stream, torch)
    plan.close()
    del plan, moms, weights
    torch.cuda.empty_cache()
    log(f"[bench] Muon step (momentum in the norm pass, weight step in the last update): {ms:.3f} ms "
        f"against {base_ms:.3f} ms for the plain plan")
    return dict(matrices=len(Gs), beta=0.95, lr=0.02, wd=0.01, weights="bf16", momentum="f32",
                ms_per_step=round(ms, 3), plain_plan_ms_per_step=round(base_ms, 3),
                overhead_ms=round(ms - base_ms, 3))


def spectral_init_row(Gs, meta, abc, T, args, stream, torch, log, base_ms):
    """The spectrum-aware initialisation (16 power steps, then the cubic as an
    extra first step) on the whole workload: ms per step against the plain
    plan's, and the polar errors of the first layer's results."""
    import paper_2505_16932_amd as pe
    plan = pe.Plan(Gs, T=T, abc=abc, compute="bf16", spectral_init=16)
    ms, _ = time_plan(plan, max(2, min(args.steps, 5)), 1, stream, torch)
    plan.launch(graph=True)
    torch.cuda.synchronize()
    n = min(7, len(Gs))
    errs = []
    if "mats" in meta:
        for k in range(n):
            errs.append(round(spec_norm_factored(plan.outs[k], *factors(meta, k), torch), 5))
    plan.close()
    del plan
    torch.cuda.empty_cache()
    log(f"[bench] spectrum-aware init: {ms:.3f} ms against {base_ms:.3f} ms; first-layer polar errors {errs}")
    return dict(power_steps=16, ms_per_step=round(ms, 3), plain_plan_ms_per_step=round(base_ms, 3),
                overhead_ms=round(ms - base_ms, 3), polar_err_first_layer=errs)


def per_head_row(Gs, abc, T, args, stream, torch, log):
    """Per-head splitting: the first layer's 4096x4096 matrices, each split into
    32 column blocks of 4096x128 (views, one grouped call), against the four
    whole matrices."""
    import paper_2505_16932_amd as pe
    sq = [G for G in Gs[:7] if G.shape[0] == G.shape[1]][:4]
    if not sq:
        return None
    heads = [h for G in sq for h in pe.split_heads(G, 32, axis=1)]
    row = dict(matrices=len(sq), shape=list(sq[0].shape), heads=len(heads), head_shape=list(heads[0].shape))
    for name, mats in (("whole", sq), ("heads", heads)):
        plan = pe.Plan(mats, T=T, abc=abc, compute="bf16")
        ms, _ = time_plan(plan, max(3, min(args.steps, 10)), 1, stream, torch)
        fl = algo_flops([tuple(m.shape) for m in mats], T)
        row[name] = dict(ms_per_call=round(ms, 3), algorithmic_tflops=round(fl / (ms * 1e-3) / 1e12, 2))
        plan.close()
        del plan
    torch.cuda.empty_cache()
    log(f"[bench] per-head split ({len(heads)} x {tuple(heads[0].shape)}): {row['heads']['ms_per_call']} ms "
        f"against {row['whole']['ms_per_call']} ms for the {len(sq)} whole matrices")
    return row


def rel_fro_np(X, ref):
    import numpy as np
    return float(np.linalg.norm(X - ref) / np.linalg.norm(ref))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="wide-batch",
                    choices=["wide-batch", "wide-layer", "gpt-small-batch", "single-4096x1024", "small-256"])
    ap.add_argument("--compute", default=None, choices=["bf16", "fp8", "f32"],
                    help="arithmetic of the timed plan: bf16 (default; f32 for small-256)")
    ap.add_argument("--fp8-steps", type=int, default=None)
    ap.add_argument("--no-fp8-variant", action="store_true",
                    help="skip the e4m3 variant timed after the main plan (wide batches)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-fast-row", action="store_true",
                    help="skip the FP32 standard-vs-fast rectangular iteration row")
    ap.add_argument("--no-extra-rows", action="store_true",
                    help="skip the Muon, spectrum-aware init and per-head rows")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--phase-reps", type=int, default=10)
    ap.add_argument("--tile", type=int, default=0, help="0 auto, 1 = 128x128, 2 = 256x256 block tile")
    ap.add_argument("--split-k", type=int, default=0,
                    help="0 auto; k >= 1 caps the Gram-side split-K factor (1 = no split)")
    ap.add_argument("--inputs", default="spectral", choices=["spectral", "gaussian"],
                    help="gaussian: iid inputs of the same shapes (profiler runs; no polar error)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a kernel of known traffic "
                         "that scales the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.compute is None:
        args.compute = "f32" if args.workload == "small-256" else "bf16"
    if args.fp8_steps is None:
        args.fp8_steps = 3 if args.compute == "fp8" else 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(matrices would be sharded across GPUs with no exchange during the iteration)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2505_16932_amd as pe

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    pe.lib()
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {nb} bytes read, {nb} bytes written")
        del src, dst
    log(f"[bench] generating workload {args.workload}")
    t0 = time.perf_counter()
    Gs, T, meta = make_workload(args.workload, torch, dev, args.inputs)
    torch.cuda.synchronize()
    log(f"[bench] {len(Gs)} matrices ready in {time.perf_counter() - t0:.1f} s")
    shapes = [tuple(G.shape) for G in Gs]
    abc = pe.coeffs(1e-3, T).abc
    stream = torch.cuda.current_stream()
    flops = algo_flops(shapes, T)
    with_err = not args.no_error and "gaussian" not in meta
    ref_idx = len(Gs) - 1           # the matrix the CPU oracle runs
    samples = {}                    # GPU results of that matrix, per variant

    def fp8_flops(steps):
        fl = 0.0
        for m, n in shapes:
            s_, L_ = min(m, n), max(m, n)
            fl += (float(s_) * s_ * L_ + float(s_) ** 3) * min(steps, T)
        return fl

    def pct_mfma(ms, steps):
        f8 = fp8_flops(steps)
        return 100.0 * ((flops - f8) / (PEAK_BF16_TFLOPS * 1e12) +
                        f8 / (PEAK_FP8_TFLOPS * 1e12)) / (ms * 1e-3)

    plan = pe.Plan(Gs, T=T, abc=abc, compute=args.compute, fp8_steps=args.fp8_steps, tile=args.tile,
                   split_k=args.split_k)
    log(f"[bench] plan ready ({args.compute}), workspace {plan.ws_bytes / 2**30:.1f} GiB")
    ms, wall_ms = time_plan(plan, args.steps, args.warmup, stream, torch)
    tflops = flops / (ms * 1e-3) / 1e12
    log(f"[bench] {ms:.3f} ms/step, {tflops:.1f} TFLOP/s (wall {wall_ms:.3f} ms/step)")

    # dominant kernel: the update X = aX + BX of a middle step, timed alone on
    # the stream it is launched on
    step = 1 if T > 2 else 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan.launch_phase(step, 3)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.phase_reps):
        plan.launch_phase(step, 3)
    e1.record(stream)
    torch.cuda.synchronize()
    upd_ms = e0.elapsed_time(e1) / args.phase_reps
    upd_tf = update_flops(shapes) / (upd_ms * 1e-3) / 1e12
    log(f"[bench] update kernel {upd_ms:.3f} ms, {upd_tf:.1f} TFLOP/s")
    # restore a valid result after the diagnostic launches
    plan.launch(graph=True)
    torch.cuda.synchronize()

    extra = {}
    if with_err:
        errs = polar_errors(plan.outs, meta, torch)
        extra["polar_err"] = err_summary(errs)
        extra["polar_err_all"] = [round(e, 5) for e in errs]
        log(f"[bench] ||X - UV^T||_2 over {len(errs)} matrices: {extra['polar_err']}")
        if "mats" in meta:
            pred = []
            for j, (U, sig, V) in enumerate(meta["templates"]):
                pred.append(round(predicted_polar_error(sig.double().cpu().numpy(), abc), 5))
            extra["polar_err_predicted_per_shape"] = pred
        samples[args.compute] = plan.outs[ref_idx].double().cpu().numpy()
    plan.close()
    del plan
    torch.cuda.empty_cache()

    if (args.workload in ("wide-batch", "wide-layer") and args.compute == "bf16"
            and not args.no_fp8_variant and "gaussian" not in meta):
        # the e4m3 variant: Gram-side products of steps 1-3 in e4m3, the rest bf16
        plan8 = pe.Plan(Gs, T=T, abc=abc, compute="fp8", fp8_steps=3, tile=args.tile)
        ms8, _ = time_plan(plan8, args.steps, args.warmup, stream, torch)
        v8 = dict(compute="fp8", fp8_steps=3, ms_per_step=round(ms8, 3),
                  tflops=round(flops / (ms8 * 1e-3) / 1e12, 2), pct_mfma_peak=round(pct_mfma(ms8, 3), 2))
        log(f"[bench] e4m3 variant {ms8:.3f} ms/step")
        plan8.launch(graph=True)
        torch.cuda.synchronize()
        if with_err:
            errs8 = polar_errors(plan8.outs, meta, torch)
            v8["polar_err"] = err_summary(errs8)
            samples["fp8"] = plan8.outs[ref_idx].double().cpu().numpy()
        extra["fp8_variant"] = v8
        plan8.close()
        del plan8
        torch.cuda.empty_cache()

    if not args.no_plain:
        # plain single-matrix bf16 path: one eager pe_polar per matrix, same schedule
        outs = [torch.empty_like(G) for G in Gs]
        for G, X in zip(Gs[:2], outs[:2]):
            pe.polar(G, T=T, abc=abc, compute="bf16", out=X, tile=args.tile)
        torch.cuda.synchronize()
        e0.record(stream)
        for G, X in zip(Gs, outs):
            pe.polar(G, T=T, abc=abc, compute="bf16", out=X, tile=args.tile)
        e1.record(stream)
        torch.cuda.synchronize()
        plain_ms = e0.elapsed_time(e1)
        extra["plain_single_matrix"] = dict(compute="bf16", ms_per_step=round(plain_ms, 3),
                                            tflops=round(flops / (plain_ms * 1e-3) / 1e12, 2),
                                            batched_speedup=round(plain_ms / ms, 3))
        if with_err:
            extra["plain_single_matrix"]["polar_err"] = err_summary(polar_errors(outs, meta, torch))
        log(f"[bench] plain bf16 path {plain_ms:.3f} ms/step")
        del outs
        torch.cuda.empty_cache()

    if args.workload in ("wide-batch", "wide-layer") and not args.no_fast_row and "mats" in meta:
        extra["fast_rect_f32"] = fast_row(Gs, meta, abc, T, args, stream, torch, log)
    if args.workload in ("wide-batch", "wide-layer") and not args.no_extra_rows and args.compute == "bf16":
        extra["muon_step"] = muon_row(Gs, abc, T, args, stream, torch, log, ms)
        extra["spectral_init"] = spectral_init_row(Gs, meta, abc, T, args, stream, torch, log, ms)
        extra["per_head"] = per_head_row(Gs, abc, T, args, stream, torch, log)

    cpu = None
    if not args.no_cpu_baseline:
        # the last three matrices (for the wide batch: three 4096x14336, about
        # 4 s each on 16 host cores); the last one is the relF sample
        idx = list(range(max(0, len(Gs) - 3), len(Gs)))
        mats64 = [Gs[i].to(torch.float64).cpu().numpy() for i in idx]
        G64 = mats64[-1]
        log(f"[bench] cpu oracle on {len(mats64)} matrices, the last {G64.shape}")
        cpu, ref = cpu_baseline(mats64, abc, T)
        log(f"[bench] cpu oracle {cpu['value']:.4f} TFLOP/s")
        if samples:
            extra["relF_vs_fp64_oracle"] = {k: float(f"{rel_fro_np(v, ref):.4e}") for k, v in samples.items()}
            extra["relF_vs_fp64_oracle"]["matrix"] = f"#{ref_idx} {G64.shape[0]}x{G64.shape[1]}"
            log(f"[bench] relF vs FP64 oracle: {extra['relF_vs_fp64_oracle']}")

    peak = PEAK_BF16_TFLOPS
    traffic = measured_traffic(args.workload, args.compute, args.tile, args.fp8_steps)
    out = {
        "metric": "polar TFLOP/s & % MFMA peak at fixed ||X-UV^T||_2, batched vs plain bf16",
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp8": "fp8e4m3+bf16", "f32": "f32"}[args.compute],
        "data": "synthetic",
        "config": {"workload": args.workload, "matrices": len(Gs), "T": T, "ell": 1e-3,
                   "compute": args.compute, "fp8_steps": args.fp8_steps, "tile": args.tile,
                   "split_k": args.split_k,
                   "shapes": sorted(set(shapes))},
        "pct_bf16_peak": round(100.0 * tflops / peak, 2),
        "pct_mfma_peak": round(pct_mfma(ms, args.fp8_steps if args.compute == "fp8" else 0), 2),
        "matrices_per_s": round(len(Gs) / (ms * 1e-3), 2),
        "dense_equivalent_tflops": round(dense_flops(shapes, T) / (ms * 1e-3) / 1e12, 2),
        "roofline": {"bound": "mfma", "achieved": round(upd_tf, 2), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(upd_tf / peak, 4),
                     "traffic": traffic["gb"] if traffic else None,
                     "traffic_unit": "GB of HBM traffic per launch (scaled FETCH_SIZE + WRITE_SIZE)",
                     "traffic_read_write_gb": [traffic["read_gb"], traffic["write_gb"]] if traffic else None,
                     "kernel": "gemm_kernel<bf16, update> (X = aX + BX)",
                     "avg_ms": round(upd_ms, 4)},
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
