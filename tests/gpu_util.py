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


def polar_error(X: np.ndarray, P: np.ndarray) -> float:
    return SP.spec_norm(np.asarray(X, dtype=np.float64) - P)


def to_np(X) -> np.ndarray:
    import torch
    return X.detach().to(torch.float64).cpu().numpy()
