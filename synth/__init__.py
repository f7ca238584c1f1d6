"""Seeded synthetic inputs shared by the tests, the oracle runs and the benchmark.

This module builds input matrices only: it holds none of the Polar Express
arithmetic (no normalisation, no polynomial, no Gram products of the method).
Matrices with a prescribed spectrum are built as G = U diag(sigma) V^T with
Haar-distributed orthonormal factors (QR of a Gaussian matrix with the signs of
diag(R) folded into Q), so that polar(G) = U V^T is known by construction.

Workloads (shapes and spectra of the method's intended use, an optimizer step
over the weight matrices of a transformer; Section 4):
* ``gaussian``       -- iid N(0, 1) entries (256 x 256, the small dense case);
* ``loguniform``     -- singular values log-uniform in [1e-4, 1] times a
                        log-uniform factor in [0.1, 10] (4096 x 1024 case);
* ``gpt_small_batch``-- 12 layers x {768x2304, 768x768, 768x3072, 3072x768},
                        sigma_i = 1/i (48 uneven matrices);
* ``wide_layer``     -- one layer of a 4096-wide model: four 4096x4096 and
                        three 4096x14336 matrices, sigma_i = 1/i; the
                        32-layer batch repeats this layer template with fresh
                        column signs and permutations of U (see ``torch_layer_batch``).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GPT_SMALL_SHAPES = [(768, 2304), (768, 768), (768, 3072), (3072, 768)]
WIDE_LAYER_SHAPES = [(4096, 4096)] * 4 + [(4096, 14336)] * 3


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar(r: np.random.Generator, m: int, k: int) -> np.ndarray:
    """m x k (m >= k) with Haar-distributed orthonormal columns."""
    Z = r.standard_normal((m, k))
    Q, R = np.linalg.qr(Z)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


@dataclass
class Synth:
    G: np.ndarray          # float64 values before any cast
    U: np.ndarray | None   # m x r
    sigma: np.ndarray | None
    V: np.ndarray | None   # n x r

    def polar(self) -> np.ndarray:
        return self.U @ self.V.T


def usv(r: np.random.Generator, m: int, n: int, sigma: np.ndarray) -> Synth:
    k = min(m, n)
    U = haar(r, m, k)
    V = haar(r, n, k)
    G = (U * sigma) @ V.T
    return Synth(G, U, np.asarray(sigma, dtype=np.float64), V)


def spectrum_loguniform(r: np.random.Generator, k: int, lo: float, hi: float) -> np.ndarray:
    return np.sort(np.exp(r.uniform(np.log(lo), np.log(hi), size=k)))[::-1].copy()


def spectrum_powerlaw(k: int, gamma: float = 1.0) -> np.ndarray:
    return np.arange(1, k + 1, dtype=np.float64) ** (-gamma)


def spectrum_clustered(r: np.random.Generator, k: int, n_centres: int, lo: float = 1e-4) -> np.ndarray:
    centres = np.exp(r.uniform(np.log(lo), 0.0, size=n_centres))
    which = r.integers(0, n_centres, size=k)
    s = centres[which] * r.uniform(0.9, 1.1, size=k)
    return np.sort(s)[::-1].copy()


def gaussian(seed: int = 1001, m: int = 256, n: int = 256) -> Synth:
    return Synth(rng(seed).standard_normal((m, n)), None, None, None)


def loguniform(seed: int = 1002, m: int = 4096, n: int = 1024,
               lo: float = 1e-4, hi: float = 1.0) -> Synth:
    r = rng(seed)
    k = min(m, n)
    sig = spectrum_loguniform(r, k, lo, hi)
    c = float(np.exp(r.uniform(np.log(0.1), np.log(10.0))))
    S = usv(r, m, n, sig)
    return Synth(S.G * c, S.U, S.sigma * c, S.V)


def powerlaw(seed: int, m: int, n: int, gamma: float = 1.0) -> Synth:
    r = rng(seed)
    return usv(r, m, n, spectrum_powerlaw(min(m, n), gamma))


def gpt_small_batch(layers: int = 12, seed0: int = 1003):
    """48 uneven matrices with sigma_i = 1/i (one seed per matrix)."""
    out = []
    k = 0
    for _ in range(layers):
        for (m, n) in GPT_SMALL_SHAPES:
            out.append(powerlaw(seed0 + k, m, n))
            k += 1
    return out


def to_bf16_values(G: np.ndarray) -> np.ndarray:
    """The float64 values of G after a round-to-nearest-even cast to bfloat16."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(G, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


# --------------------------------------------------------------------------
# device-side generation for the large batch (torch only supplies the RNG,
# QR and products used to build inputs)
# --------------------------------------------------------------------------
def torch_haar(gen, m: int, k: int, device):
    import torch
    Z = torch.randn((m, k), generator=gen, device=device, dtype=torch.float32)
    Q, R = torch.linalg.qr(Z)
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d


def torch_layer_batch(layers: int, seed: int, device, dtype=None, shapes=None, gamma: float = 1.0):
    """Matrices of a ``layers``-deep model built from one Haar layer template.

    Layer 0's factors U_j, V_j come from QR; every later layer uses
    U_j[:, perm] * signs with a fresh permutation and sign vector, which is
    again a matrix with orthonormal columns, so each G = U' diag(sigma) V^T has
    the prescribed spectrum and known polar factor U' V^T.  Returns a list of
    (G, perm, signs, template_index) and the template factors.
    """
    import torch
    dtype = dtype or torch.bfloat16
    shapes = shapes or WIDE_LAYER_SHAPES
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    templates = []
    for (m, n) in shapes:
        k = min(m, n)
        U = torch_haar(gen, m, k, device)
        V = torch_haar(gen, n, k, device)
        sig = torch.arange(1, k + 1, device=device, dtype=torch.float32) ** (-gamma)
        templates.append((U, sig, V))
    mats = []
    for layer in range(layers):
        for j, (U, sig, V) in enumerate(templates):
            k = U.shape[1]
            if layer == 0:
                perm = torch.arange(k, device=device)
                signs = torch.ones(k, device=device)
            else:
                perm = torch.randperm(k, generator=gen, device=device)
                signs = torch.randint(0, 2, (k,), generator=gen, device=device).float() * 2 - 1
            Up = U[:, perm] * signs
            G = ((Up * sig) @ V.T).to(dtype)
            mats.append((G, perm, signs, j))
    return mats, templates
