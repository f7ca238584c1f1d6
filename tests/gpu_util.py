"""Helpers shared by the GPU parity tests: seeded inputs on the device and
oracle references computed from the exact values the device received."""
import numpy as np

import synth
from oracle import iteration as OI
from oracle import schedule as OS
from oracle import spectral as SP


def device_input(G64: np.ndarray, dtype):
    """Cast float64 values to the device dtype; return (tensor, float64 values read back)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(G64, dtype=np.float32)).to(dtype)
    vals = t.to(torch.float64).numpy()
    return t.to("cuda"), vals


def oracle_schedule(T: int, ell: float = 1e-3) -> np.ndarray:
    return OS.greedy_schedule(ell, T).abc


def oracle_same_iteration(vals: np.ndarray, abc) -> np.ndarray:
    return OI.polar_express(vals, abc)


def relf(X, ref) -> float:
    return OI.rel_fro(X, ref)


def tile_relf(X, ref, bt: int = 256) -> float:
    """Largest block error over the bt x bt blocks of the output: the block's
    error ||X_b - ref_b||_F relative to the larger of ||ref_b||_F and the
    block's share of the whole reference, ||ref||_F sqrt(|b| / |ref|) (thin
    edge blocks and blocks with little content are measured against the
    matrix-average scale, so an error confined to one block shows up while a
    near-zero block does not blow up)."""
    X = np.asarray(X, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    tot = float(np.linalg.norm(ref))
    if tot == 0:
        return float(np.linalg.norm(X))
    worst = 0.0
    for i in range(0, ref.shape[0], bt):
        for j in range(0, ref.shape[1], bt):
            r = ref[i:i + bt, j:j + bt]
            den = max(float(np.linalg.norm(r)), tot * np.sqrt(r.size / ref.size))
            worst = max(worst, float(np.linalg.norm(X[i:i + bt, j:j + bt] - r)) / den)
    return worst


def polar_error(X: np.ndarray, P: np.ndarray) -> float:
    return SP.spec_norm(np.asarray(X, dtype=np.float64) - P)


def to_np(X) -> np.ndarray:
    import torch
    return X.detach().to(torch.float64).cpu().numpy()
