"""Autotuner of the block tile per shape class and call regime.

For each shape class (precision, s bucket, aspect bucket) and regime -- "x1",
a call with one matrix (below the library's 3e12 FLOP-per-step batch
threshold), and "xN", a batch of ~1.5e13 FLOP per step -- it builds a batch
of that class, times
whole plan launches (hipGraph replays, HIP events on the launch stream) with
each compiled tile (1 = 128 x 128, 2 = 256 x 256), and writes
"<shape-class>_<regime> <tile-id>" lines to a table that pe_tile_table_load()
reads (the binding loads tile_table.txt next to the library when it exists).

    python -m paper_2505_16932_amd.autotune [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import ctypes
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tile_table.txt")

S_BUCKETS = (256, 512, 1024, 2048, 4096)
ASPECTS = (1, 3, 8)


def representative(s_bucket: int, aspect: int):
    """An m x n shape whose class is (s_bucket, aspect bucket): wide, s = m."""
    return s_bucket, s_bucket * aspect


def time_plan(pe, torch, shape, count, tile, compute, reps=5):
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    Gs = [torch.randn(shape, generator=g, device="cuda").to(torch.bfloat16) for _ in range(count)]
    plan = pe.Plan(Gs, T=5, compute=compute, tile=tile)
    plan.launch(graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st = torch.cuda.current_stream()
    e0.record(st)
    for _ in range(reps):
        plan.launch(graph=True)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    plan.close()
    del Gs
    return ms


def batch_count(regime: str, m: int, n: int) -> int:
    """Matrices of one timed call: 1 for x1; for xN enough for ~1.5e13
    algorithmic FLOP per step (at least 2), within about 40 GB of inputs,
    outputs and workspace (~16 bytes per element)."""
    if regime == "x1":
        return 1
    s, Lx = min(m, n), max(m, n)
    flops = 5 * (3.0 * s * s * Lx + float(s) ** 3)
    by_mem = int(40e9 // (16.0 * m * n))
    return int(max(2, min(64, by_mem, round(1.5e13 / flops))))


def tune(out_path=DEFAULT_TABLE, compute="bf16", quick=False, log=print):
    import torch
    import paper_2505_16932_amd as pe
    L = pe.lib()
    lines = [f"# block tile per shape class and call regime (_x1: one matrix, _xN: a batch), "
             f"{compute}, measured by paper_2505_16932_amd.autotune",
             "# class tile ms_tile1 ms_tile2 (per call)"]
    rows = []
    buckets = S_BUCKETS[:3] if quick else S_BUCKETS
    for sb in buckets:
        for a in ASPECTS:
            m, n = representative(sb, a)
            cls = L.pe_shape_class(pe.COMPUTE[compute], m, n).decode()
            for regime in ("x1", "xN"):
                count = batch_count(regime, m, n)
                t1 = time_plan(pe, torch, (m, n), count, 1, compute)
                t2 = time_plan(pe, torch, (m, n), count, 2, compute)
                best = 1 if t1 <= t2 else 2
                key = f"{cls}_{regime}"
                rows.append((key, best, t1, t2))
                log(f"[autotune] {key}: {count} x {m}x{n}  tile128 {t1:.3f} ms  tile256 {t2:.3f} ms -> {best}")
                lines.append(f"{key} {best}  # {t1:.4f} {t2:.4f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--compute", default="bf16")
    ap.add_argument("--quick", action="store_true")
    a = ap.parse_args()
    tune(a.out, a.compute, a.quick, log=lambda s: print(s, flush=True))
    return 0


if __name__ == "__main__":
    sys.exit(main())
