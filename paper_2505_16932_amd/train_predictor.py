"""Train the l-predictor on the device and save its weights next to the library.

    python -m paper_2505_16932_amd.train_predictor [--samples 200000] [--T 5]
        [--epochs 30] [--out paper_2505_16932_amd/predictor_T5]

Training data are (shape, spectrum) samples from ``learned.sample_spectrum``
(features and labels need only the normalised spectrum, by the identity of
Appendix C), built on the host in worker processes; the network is trained
with the library's own forward/backward/Adam kernels (``learned.train``), then
evaluated on a held-out set.  Writes <out>.npy (the 5768 FP32 parameters in
the layout of pe.h) and <out>.json (how they were made and the held-out
figures).  The binding's ``load_predictor`` reads them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _chunk(args):
    n, seed, T = args
    from paper_2505_16932_amd import learned as PL
    return PL.build_dataset(n, seed, T)


def build_parallel(n: int, seed: int, T: int, workers: int):
    """build_dataset over ``workers`` processes, chunk k seeded seed * 1000 + k."""
    from multiprocessing import get_context
    per = (n + workers - 1) // workers
    jobs = [(min(per, n - k * per), seed * 1000 + k, T) for k in range(workers) if n - k * per > 0]
    with get_context("spawn").Pool(len(jobs)) as pool:
        parts = pool.map(_chunk, jobs)
    F = np.concatenate([p[0] for p in parts])
    Y = np.concatenate([p[1] for p in parts])
    E = np.concatenate([p[2] for p in parts])
    return F, Y, E


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=200000)
    ap.add_argument("--heldout", type=int, default=20000)
    ap.add_argument("--T", type=int, default=5)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=1005)
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--out", default=os.path.join(HERE, "predictor_T5"))
    a = ap.parse_args(argv)
    import torch

    from paper_2505_16932_amd import learned as PL
    t0 = time.time()
    F, Y, E = build_parallel(a.samples, a.seed, a.T, a.workers)
    Fh, Yh, Eh = build_parallel(a.heldout, a.seed + 1, a.T, a.workers)
    t_data = time.time() - t0
    print(f"[train] {len(Y)} training and {len(Yh)} held-out spectra in {t_data:.1f} s; "
          f"label counts {np.bincount(Y, minlength=8).tolist()}", flush=True)
    t1 = time.time()
    params = PL.train(F, Y, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed,
                      log=lambda s: print("[train]", s, flush=True))
    torch.cuda.synchronize()
    t_train = time.time() - t1
    res = PL.evaluate(params, Fh, Eh, T=a.T, Y=Yh)
    tr = PL.evaluate(params, F[:20000], E[:20000], T=a.T, Y=Y[:20000])
    theta = params.cpu().numpy().astype(np.float32)
    np.save(a.out + ".npy", theta, allow_pickle=False)
    meta = dict(
        T=a.T, classes=[[l, k] for l, k in PL.CLASS_TABLE], fixed_class=PL.FIXED_CLASS,
        samples=len(Y), heldout=len(Yh), seed=a.seed, epochs=a.epochs, batch=a.batch, lr=a.lr,
        label_rule="fewest steps within the fixed class's error, then the smallest error",
        label_counts=np.bincount(Y, minlength=8).tolist(),
        heldout_metrics={k: v for k, v in res.items() if k != "classes"},
        train_metrics={k: v for k, v in tr.items() if k != "classes"},
        heldout_class_counts=np.bincount(res["classes"], minlength=8).tolist(),
        seconds=dict(data=round(t_data, 1), train=round(t_train, 1)),
        trained_with="pe_mlp_train_step (device kernels)",
    )
    with open(a.out + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    print(f"[train] held-out: {meta['heldout_metrics']}", flush=True)
    print(f"[train] wrote {a.out}.npy and {a.out}.json", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
