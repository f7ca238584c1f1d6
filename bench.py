#!/usr/bin/env python3
"""Polar Express throughput on one MI355X.

One step = one pass of the whole method (norm + T polynomial steps) over every
matrix of the workload, through a plan (grouped launches captured as a
hipGraph).  Inputs are synthetic, seeded, resident in HBM before timing.

Workloads:
  wide-batch        32-layer 4096-wide model: per layer four 4096x4096 and three
                    4096x14336 bf16 matrices (224), sigma_i = 1/i, Haar singular
                    vectors, T = 5; the Gram-side products of steps 1-3 in e4m3
                    with per-tensor scales, everything else bf16    (default)
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


def polar_factor(meta, idx, torch):
    """U' V^T of matrix idx (known by construction)."""
    if "polar" in meta:
        return meta["polar"]
    if "mats" in meta:
        G, perm, signs, j = meta["mats"][idx]
        U, sig, V = meta["templates"][j]
        return (U[:, perm] * signs) @ V.T
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


def cpu_baseline(G_cpu64, abc, T):
    """The FP64 oracle on the host cores, on one matrix of the workload."""
    import numpy as np
    from oracle import iteration as OI
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    t0 = time.perf_counter()
    OI.polar_express(G_cpu64, abc)
    dt = time.perf_counter() - t0
    m, n = G_cpu64.shape
    fl = algo_flops([(m, n)], T)
    return dict(value=fl / dt / 1e12, unit="TFLOP/s", cores=int(cores), kind="oracle",
                sample=f"1 of the workload's matrices ({m}x{n}), T={T}, FP64 NumPy, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="wide-batch",
                    choices=["wide-batch", "wide-layer", "gpt-small-batch", "single-4096x1024", "small-256"])
    ap.add_argument("--compute", default=None, choices=["bf16", "fp8", "f32"],
                    help="default: fp8 (Gram-side steps 1-3) for wide-batch, bf16 otherwise")
    ap.add_argument("--fp8-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--phase-reps", type=int, default=10)
    ap.add_argument("--tile", type=int, default=0, help="0 auto, 1 = 128x128, 2 = 256x256 block tile")
    ap.add_argument("--inputs", default="spectral", choices=["spectral", "gaussian"],
                    help="gaussian: iid inputs of the same shapes (profiler runs; no polar error)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a kernel of known traffic "
                         "that scales the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.compute is None:
        args.compute = "fp8" if args.workload == "wide-batch" else "bf16"
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

    plan = pe.Plan(Gs, T=T, abc=abc, compute=args.compute, fp8_steps=args.fp8_steps, tile=args.tile)
    log(f"[bench] plan ready, workspace {plan.ws_bytes / 2**30:.1f} GiB")
    for _ in range(args.warmup):
        plan.launch(graph=True)
    torch.cuda.synchronize()
    log("[bench] warmup done")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.launch(graph=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1) / args.steps
    flops = algo_flops(shapes, T)
    tflops = flops / (ms * 1e-3) / 1e12
    log(f"[bench] {ms:.3f} ms/step, {tflops:.1f} TFLOP/s (wall {wall / args.steps * 1e3:.3f} ms/step)")

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
    if not args.no_error and "gaussian" not in meta:
        errs = []
        for idx in sorted(set([0, min(4, len(Gs) - 1)])):
            P = polar_factor(meta, idx, torch).float()
            errs.append(spec_norm_gpu(plan.outs[idx].float() - P, torch))
        extra["polar_err_sampled"] = [round(e, 5) for e in errs]
        log(f"[bench] ||X - UV^T||_2 on sampled matrices: {errs}")

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
                                            tflops=round(flops / (plain_ms * 1e-3) / 1e12, 2))
        if not args.no_error and "gaussian" not in meta:
            perr = []
            for idx in sorted(set([0, min(4, len(Gs) - 1)])):
                P = polar_factor(meta, idx, torch).float()
                perr.append(round(spec_norm_gpu(outs[idx].float() - P, torch), 5))
            extra["plain_single_matrix"]["polar_err_sampled"] = perr
        log(f"[bench] plain bf16 path {plain_ms:.3f} ms/step")
        del outs

    cpu = None
    if not args.no_cpu_baseline:
        idx = len(Gs) - 1
        G64 = Gs[idx].to(torch.float64).cpu().numpy()
        log(f"[bench] cpu oracle on {G64.shape}")
        cpu = cpu_baseline(G64, abc, T)
        log(f"[bench] cpu oracle {cpu['value']:.4f} TFLOP/s")

    peak = PEAK_BF16_TFLOPS
    traffic = measured_traffic(args.workload, args.compute, args.tile, args.fp8_steps)
    # MFMA-peak fraction with each product at its own precision's dense peak
    fp8_fl = 0.0
    if args.compute == "fp8":
        for m, n in shapes:
            s_, L_ = min(m, n), max(m, n)
            fp8_fl += (float(s_) * s_ * L_ + float(s_) ** 3) * min(args.fp8_steps, T)
    pct_mfma = 100.0 * ((flops - fp8_fl) / (PEAK_BF16_TFLOPS * 1e12) +
                        fp8_fl / (PEAK_FP8_TFLOPS * 1e12)) / (ms * 1e-3)
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
                   "shapes": sorted(set(shapes))},
        "pct_bf16_peak": round(100.0 * tflops / peak, 2),
        "pct_mfma_peak": round(pct_mfma, 2),
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
    plan.close()


if __name__ == "__main__":
    main()
