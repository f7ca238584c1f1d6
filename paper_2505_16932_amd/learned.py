"""Training data and training loop of the l-predictor.

The paper guesses l = 1e-3 for every matrix (Section 3.3).  The predictor
picks, per matrix, one of eight schedules from moments of the step-1 Gram
matrix; a schedule is a pair (l, T') from CLASS_TABLE -- the greedy schedule
for l run for T' <= T steps, the device skipping the matrix's later steps --
so that matrices whose spectrum allows it finish early.  Because the polar
error of a polynomial iteration depends only on the normalised spectrum
(Appendix C: ||polar(M) - p(M)||_2 = max_i |1 - p(sigma_i)|), training
samples are (shape, spectrum) pairs:

* features: the 16 values the selection kernel computes on the device from
  s, L and m_k = sum_i sigma_hat_i^(2k), k = 1..4 (same formula, float64 here);
* label: among the classes whose error max_i |1 - phi(sigma_hat_i)| does not
  exceed the fixed class's (l = 1e-3, all T steps), the one with the fewest
  steps, then the smallest error.

Spectrum families follow the intended use (weight-gradient-like matrices):
log-uniform on [10^-k, 1] (k ~ U[1, 6]), power law i^-gamma (gamma ~ U[0.3, 2]),
and 1-4 clusters (log-uniform centres, +-10% spread); shapes m, n log-uniform
in [128, 2048] with aspect ratio at most 8.  The network is trained by the
library's own device kernels (pe_mlp_train_step).
"""
from __future__ import annotations

import numpy as np

from . import CLASSES, FEATURES, FIXED_CLASS, MLP_PARAMS, MLPTrainer, coeffs

# (l, T'), T' = None: all T steps; must match the library's class table
CLASS_TABLE = ((1e-1, 2), (1e-1, 3), (3e-2, 3), (1e-2, 4), (1e-3, None), (3e-3, 4), (3e-4, None),
               (1e-4, None))
CLASS_ELL = tuple(c[0] for c in CLASS_TABLE)


def class_steps(T: int) -> np.ndarray:
    return np.array([T if k is None else min(T, k) for _, k in CLASS_TABLE])


def class_schedules(T: int):
    return [coeffs(l, int(k)).abc for (l, _), k in zip(CLASS_TABLE, class_steps(T))]


def _phi(abc_list, x):
    y = x
    for a, b, c in abc_list:
        y2 = y * y
        y = y * (a + y2 * (b + c * y2))
    return y


def features(s: int, L: int, m) -> np.ndarray:
    """The selection kernel's 16 features (float64)."""
    m1, m2, m3, m4 = (max(float(v), 1e-300) for v in m)
    ls, lL = np.log(max(s, 1)), np.log(max(L, 1))
    l1, l2, l3, l4 = np.log(m1), np.log(m2), np.log(m3), np.log(m4)
    den = max(ls, 1e-3)
    return np.array([ls / 8.0, lL / 8.0, lL - ls, l1, l2 / 4.0, l3 / 8.0, l4 / 8.0,
                     (2 * l1 - l2) / den, (2 * l2 - l4) / den, l1 + l3 - 2 * l2,
                     l2 + l4 - 2 * l3, l4 / 8.0 - l1 / 2.0, (2 * l1 - l2) / 8.0,
                     (2 * l2 - l4) / 8.0, ls - (2 * l1 - l2), 1.0])


def normalised(sigma):
    sigma = np.asarray(sigma, dtype=np.float64)
    return sigma / (1.01 * np.sqrt(np.sum(sigma * sigma)) + 1e-7)


def sample_spectrum(rng: np.random.Generator):
    """(m, n, sigma, family) of one synthetic training matrix."""
    while True:
        m = int(np.exp(rng.uniform(np.log(128), np.log(2048))))
        n = int(np.exp(rng.uniform(np.log(128), np.log(2048))))
        if max(m, n) <= 8 * min(m, n):
            break
    k = min(m, n)
    fam = int(rng.integers(0, 3))
    if fam == 0:
        lo = 10.0 ** -rng.uniform(1, 6)
        sig = np.exp(rng.uniform(np.log(lo), 0.0, k))
    elif fam == 1:
        sig = np.arange(1, k + 1, dtype=np.float64) ** -rng.uniform(0.3, 2.0)
    else:
        nc = int(rng.integers(1, 5))
        centres = np.exp(rng.uniform(np.log(1e-4), 0.0, nc))
        sig = centres[rng.integers(0, nc, k)] * rng.uniform(0.9, 1.1, k)
    return m, n, np.sort(sig)[::-1], fam


def label_errors(sig_hat, scheds):
    return np.array([np.max(np.abs(1.0 - _phi(abc, sig_hat))) for abc in scheds])


def best_class(errs, steps, rtol=1e-9):
    """Fewest steps within the fixed class's error, then the smallest error."""
    errs = np.asarray(errs)
    ok = [c for c in range(len(errs)) if errs[c] <= errs[FIXED_CLASS] * (1 + rtol) + 1e-15]
    return min(ok, key=lambda c: (steps[c], errs[c], c))


def build_dataset(n: int, seed: int, T: int):
    """features [n x 16] float32, labels [n] int32, per-class errors [n x 8]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scheds = class_schedules(T)
    steps = class_steps(T)
    F = np.zeros((n, FEATURES), dtype=np.float32)
    Y = np.zeros(n, dtype=np.int32)
    E = np.zeros((n, CLASSES))
    for i in range(n):
        m, k, sig, _ = sample_spectrum(rng)
        sh = normalised(sig)
        s2 = sh * sh
        mom = (np.sum(s2), np.sum(s2 ** 2), np.sum(s2 ** 3), np.sum(s2 ** 4))
        F[i] = features(min(m, k), max(m, k), mom)
        E[i] = label_errors(sh, scheds)
        Y[i] = best_class(E[i], steps)
    return F, Y, E


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases, in the flat layout of pe.h."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = [rng.standard_normal((16, 64)) * np.sqrt(2 / 16), np.zeros(64),
             rng.standard_normal((64, 64)) * np.sqrt(2 / 64), np.zeros(64),
             rng.standard_normal((64, 8)) * np.sqrt(2 / 64), np.zeros(8)]
    theta = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert theta.size == MLP_PARAMS
    return theta


def train(F, Y, epochs: int = 30, batch: int = 1024, lr: float = 3e-3, seed: int = 0,
          device="cuda", log=None):
    """Mini-batch Adam with the device kernels; returns the parameter tensor."""
    import torch
    params = torch.from_numpy(init_params(seed)).to(device)
    tr = MLPTrainer(params, batch)
    Ft = torch.from_numpy(np.ascontiguousarray(F, dtype=np.float32)).to(device)
    Yt = torch.from_numpy(np.ascontiguousarray(Y, dtype=np.int32)).to(device)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    n = F.shape[0]
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(device)
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            loss = tr.train_step(Ft[idx].contiguous(), Yt[idx].contiguous(), lr_ep)
            tot += float(loss.item()) if (cnt % 20 == 0) else 0.0
            cnt += 1
        if log:
            log(f"epoch {ep} lr {lr_ep:.2e}")
    torch.cuda.synchronize()
    return params


def evaluate(params, F, E, T: int, Y=None, device="cuda"):
    """Steps and per-sample error of the chosen classes against the fixed class."""
    import torch
    from . import mlp_forward
    logits = mlp_forward(params, torch.from_numpy(np.ascontiguousarray(F, dtype=np.float32)).to(device))
    cls = logits.argmax(dim=1).cpu().numpy()
    steps = class_steps(T)
    chosen = E[np.arange(len(cls)), cls]
    fixed = E[:, FIXED_CLASS]
    worse = chosen > fixed * (1 + 1e-9) + 1e-15
    return dict(mean_steps=float(steps[cls].mean()), fixed_steps=float(T),
                mean_chosen=float(chosen.mean()), mean_fixed=float(fixed.mean()),
                frac_fewer_steps=float(np.mean(steps[cls] < T)),
                frac_better=float(np.mean(chosen < fixed - 1e-12)),
                frac_worse=float(np.mean(worse)),
                mean_excess_when_worse=float((chosen - fixed)[worse].mean()) if worse.any() else 0.0,
                accuracy=float(np.mean(cls == Y)) if Y is not None else None, classes=cls)
