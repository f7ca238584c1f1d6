"""Autotuner of the block tile per shape class.

For each shape class (precision, s bucket, aspect bucket) it builds a batch of
representative matrices, times whole plan launches (hipGraph replays, HIP
events on the launch stream) with each compiled tile (1 = 128 x 128,
2 = 256 x 256), and writes "<shape-class> <tile-id>" lines to a table that
pe_tile_table_load() reads (the binding loads tile_table.txt next to the
library when it exists).

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


def tune(out_path=DEFAULT_TABLE, compute="bf16", quick=False, log=print):
    import torch
    import paper_2505_16932_amd as pe
    L = pe.lib()
    lines = [f"# block tile per shape class, {compute}, measured by paper_2505_16932_amd.autotune",
             "# class tile ms_tile1 ms_tile2"]
    rows = []
    buckets = S_BUCKETS[:3] if quick else S_BUCKETS
    for sb in buckets:
        for a in ASPECTS:
            m, n = representative(sb, a)
            s, Lx = min(m, n), max(m, n)
            flops = 5 * (3.0 * s * s * Lx + float(s) ** 3)
            count = int(max(1, min(64, round(4e11 / flops))))
            cls = L.pe_shape_class(pe.COMPUTE[compute], m, n).decode()
            t1 = time_plan(pe, torch, (m, n), count, 1, compute)
            t2 = time_plan(pe, torch, (m, n), count, 2, compute)
            best = 1 if t1 <= t2 else 2
            rows.append((cls, best, t1, t2))
            log(f"[autotune] {cls}: {count} x {m}x{n}  tile128 {t1:.3f} ms  tile256 {t2:.3f} ms -> {best}")
            lines.append(f"{cls} {best}  # {t1:.4f} {t2:.4f}")
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
