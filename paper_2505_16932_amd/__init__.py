"""Python binding of the gfx950 Polar Express library (libpe.so, C ABI in include/pe.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels (or, for the coefficient schedule, its host FP64 code).  PyTorch
supplies device memory (inputs, outputs, workspace) and the current stream.

    import paper_2505_16932_amd as pe
    abc = pe.coeffs(1e-3, 5).abc                       # offline stage, FP64
    X = pe.polar(G, T=5)                               # one matrix
    Xs = pe.polar_batched([G1, G2, G3], T=5)           # grouped launches
    plan = pe.Plan(Gs, T=5); plan.launch(graph=True)   # tables once + hipGraph

The library file must have been built (``paper_2505_16932_amd.build``); there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

__all__ = ["coeffs", "coeffs_cubic", "split_heads", "load_predictor", "polar", "polar_batched", "polar_noalloc", "muon_step", "Plan", "workspace_size", "lib", "PEError",
           "COMPUTE", "LIB_PATH"]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpe.so")

PE_F32, PE_BF16 = 0, 1
COMPUTE = {"f32": 0, "bf16": 1, "fp8": 2}
STATUS = {0: "PE_OK", 1: "PE_EINVAL", 2: "PE_EUNSUPPORTED", 3: "PE_ENOCONV",
          4: "PE_EWORKSPACE", 5: "PE_EHIP"}


class PEError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = f"{where}: {STATUS.get(status, status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


class CoeffOpts(ctypes.Structure):
    _fields_ = [("cushion", ctypes.c_double), ("safety", ctypes.c_double),
                ("safety_on_last", ctypes.c_int32)]


class Matrix(ctypes.Structure):
    _fields_ = [("G", ctypes.c_void_p), ("X", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("n", ctypes.c_int64), ("ldg", ctypes.c_int64), ("ldx", ctypes.c_int64),
                ("g_dtype", ctypes.c_int32), ("x_dtype", ctypes.c_int32),
                ("M", ctypes.c_void_p), ("ldm", ctypes.c_int64), ("W", ctypes.c_void_p),
                ("ldw", ctypes.c_int64), ("w_dtype", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("abc", ctypes.POINTER(ctypes.c_double)),
                ("compute", ctypes.c_int32), ("fp8_steps", ctypes.c_int32),
                ("norm_mode", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("predictor", ctypes.c_void_p), ("force_class", ctypes.c_int32),
                ("fallback_tau", ctypes.c_float), ("split_k", ctypes.c_int32),
                ("fast_restart", ctypes.c_int32), ("fast_eps", ctypes.c_float),
                ("muon_beta", ctypes.c_float), ("muon_lr", ctypes.c_float), ("muon_wd", ctypes.c_float),
                ("spectral_init", ctypes.c_int32)]


MLP_PARAMS = 5768
CLASSES = 8
FIXED_CLASS = 4
FEATURES = 16


_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded libpe.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2505_16932_amd.build` (no fallback path exists)")
        # torch ships its own HIP runtime; import it first so that the library's
        # libamdhip64.so.7 dependency resolves to that same loaded runtime
        # (two HIP runtimes in one process do not share devices)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.pe_coeffs.restype = ctypes.c_int
        L.pe_coeffs.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.POINTER(CoeffOpts),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
        L.pe_coeffs_cubic.restype = ctypes.c_int
        L.pe_coeffs_cubic.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.POINTER(CoeffOpts),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
        L.pe_coeff_opts_default.restype = None
        L.pe_coeff_opts_default.argtypes = [ctypes.POINTER(CoeffOpts)]
        L.pe_workspace_size.restype = ctypes.c_size_t
        L.pe_workspace_size.argtypes = [ctypes.c_int32, ctypes.POINTER(Matrix), ctypes.POINTER(Opts)]
        L.pe_polar.restype = ctypes.c_int
        L.pe_polar.argtypes = [ctypes.POINTER(Matrix), ctypes.POINTER(Opts), ctypes.c_void_p,
                               ctypes.c_size_t, ctypes.c_void_p]
        L.pe_polar_noalloc.restype = ctypes.c_int
        L.pe_polar_noalloc.argtypes = [ctypes.POINTER(Matrix), ctypes.POINTER(Opts), ctypes.c_void_p]
        L.pe_polar_batched.restype = ctypes.c_int
        L.pe_polar_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(Matrix), ctypes.POINTER(Opts),
                                       ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.pe_plan_create.restype = ctypes.c_int
        L.pe_plan_create.argtypes = [ctypes.c_int32, ctypes.POINTER(Matrix), ctypes.POINTER(Opts),
                                     ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_void_p)]
        L.pe_plan_launch.restype = ctypes.c_int
        L.pe_plan_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        L.pe_plan_launch_phase.restype = ctypes.c_int
        L.pe_plan_launch_phase.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_void_p]
        L.pe_plan_destroy.restype = ctypes.c_int
        L.pe_plan_destroy.argtypes = [ctypes.c_void_p]
        L.pe_quantize_e4m3.restype = ctypes.c_int
        L.pe_quantize_e4m3.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_float, ctypes.c_void_p]
        L.pe_plan_selection.restype = ctypes.c_int
        L.pe_plan_selection.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.pe_mlp_workspace_size.restype = ctypes.c_size_t
        L.pe_mlp_workspace_size.argtypes = [ctypes.c_int32]
        L.pe_mlp_forward.restype = ctypes.c_int
        L.pe_mlp_forward.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p]
        L.pe_mlp_grad.restype = ctypes.c_int
        L.pe_mlp_grad.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p]
        L.pe_mlp_train_step.restype = ctypes.c_int
        L.pe_mlp_train_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int32, ctypes.c_float, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.pe_tile_count.restype = ctypes.c_int32
        L.pe_tile_name.restype = ctypes.c_char_p
        L.pe_tile_name.argtypes = [ctypes.c_int32]
        L.pe_tile_table_load.restype = ctypes.c_int
        L.pe_tile_table_load.argtypes = [ctypes.c_char_p]
        L.pe_status_string.restype = ctypes.c_char_p
        L.pe_status_string.argtypes = [ctypes.c_int]
        L.pe_last_error.restype = ctypes.c_char_p
        L.pe_shape_class.restype = ctypes.c_char_p
        L.pe_shape_class.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64]
        table = os.path.join(HERE, "tile_table.txt")
        if os.path.exists(table) and os.environ.get("PE_TILE_TABLE", "1") != "0":
            _check(L.pe_tile_table_load(table.encode()), "pe_tile_table_load")
        _LIB = L
    return _LIB


def _invalid(L, count, mats, o):
    """pe_workspace_size returned 0: raise with the status the call itself
    reports (argument checks run before anything touches the device)."""
    st = L.pe_polar_batched(count, mats, ctypes.byref(o), None, 0, None)
    _check(st if st not in (0, 4) else 1, "argument check")


def _check(st: int, where: str):
    if st != 0:
        detail = lib().pe_last_error().decode() if st in (4, 5) else ""
        raise PEError(st, where, detail)


# ------------------------------------------------------------------ offline
@dataclass
class Coeffs:
    abc: np.ndarray       # (T, 3)
    bounds: np.ndarray    # (T+1, 2): l_t, u_t
    err_bound: float      # 1 - l_{T+1}
    iters: np.ndarray     # (T,) Remez exchanges (0 = Newton-Schulz step)


def coeffs(ell: float = 1e-3, T: int = 5, cushion: float | None = None, safety: float | None = None,
           safety_on_last: bool = True) -> Coeffs:
    """Greedy minimax schedule (pe_coeffs, host FP64)."""
    L = lib()
    o = CoeffOpts()
    L.pe_coeff_opts_default(ctypes.byref(o))
    if cushion is not None:
        o.cushion = cushion
    if safety is not None:
        o.safety = safety
    o.safety_on_last = 1 if safety_on_last else 0
    abc = np.zeros(3 * T)
    bounds = np.zeros(2 * (T + 1))
    err = ctypes.c_double(0.0)
    iters = np.zeros(T, dtype=np.int32)
    dp = ctypes.POINTER(ctypes.c_double)
    st = L.pe_coeffs(float(ell), int(T), ctypes.byref(o), abc.ctypes.data_as(dp),
                     bounds.ctypes.data_as(dp), ctypes.byref(err),
                     iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    _check(st, "pe_coeffs")
    return Coeffs(abc.reshape(T, 3), bounds.reshape(T + 1, 2), err.value, iters)


def coeffs_cubic(ell: float = 1e-3, T: int = 8, safety: float | None = None,
                 safety_on_last: bool = True) -> Coeffs:
    """Degree-3 greedy schedule (pe_coeffs_cubic, host FP64): (a, b, 0) triples."""
    L = lib()
    o = CoeffOpts()
    L.pe_coeff_opts_default(ctypes.byref(o))
    if safety is not None:
        o.safety = safety
    o.safety_on_last = 1 if safety_on_last else 0
    abc = np.zeros(3 * T)
    bounds = np.zeros(2 * (T + 1))
    err = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(L.pe_coeffs_cubic(float(ell), int(T), ctypes.byref(o), abc.ctypes.data_as(dp),
                             bounds.ctypes.data_as(dp), ctypes.byref(err)), "pe_coeffs_cubic")
    return Coeffs(abc.reshape(T, 3), bounds.reshape(T + 1, 2), err.value, np.zeros(T, dtype=np.int32))


def split_heads(G, heads: int, axis: int = 1):
    """Views of a weight gradient split into ``heads`` equal slices along
    ``axis`` (Appendix G, application to Muon: each attention head's block of
    [W_Q | W_K | W_V] or W_O as its own matrix), for pe_polar_batched: no
    copies, the views keep G's leading dimension."""
    size = G.shape[axis]
    if size % heads:
        raise ValueError("the split axis must divide into the heads")
    w = size // heads
    return [G.narrow(axis, h * w, w) for h in range(heads)]


# ------------------------------------------------------------------- online
def _dtype_code(dt):
    import torch
    if dt == torch.float32:
        return PE_F32
    if dt == torch.bfloat16:
        return PE_BF16
    raise TypeError(f"unsupported dtype {dt} (float32 or bfloat16)")


def _matrix(G, X, M=None, W=None) -> Matrix:
    """Descriptor of one matrix: input G, output X (or None when W is given),
    and the optional Muon momentum M (FP32, updated in place) and weights W."""
    import torch
    for name, t in (("G", G), ("X", X), ("M", M), ("W", W)):
        if t is None:
            continue
        if t.dim() != 2 or tuple(t.shape) != tuple(G.shape):
            raise ValueError(f"{name} must be 2-D of G's shape")
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if G.numel() > 0 and t.stride(1) != 1:
            raise ValueError(f"rows of {name} must be contiguous")
    if X is None and W is None:
        raise ValueError("an output X or weights W are needed")
    if M is not None and M.dtype != torch.float32:
        raise TypeError("the momentum M must be float32")
    m, n = G.shape

    def ld(t):
        return max(t.stride(0), n) if t is not None else 0

    return Matrix(G.data_ptr(), X.data_ptr() if X is not None else None, m, n, ld(G), ld(X),
                  _dtype_code(G.dtype), _dtype_code(X.dtype) if X is not None else 0,
                  M.data_ptr() if M is not None else None, ld(M),
                  W.data_ptr() if W is not None else None, ld(W),
                  _dtype_code(W.dtype) if W is not None else 0)


def _opts(T, abc, compute, fp8_steps, norm_mode, tile, predictor=None, force_class=-1,
          fallback_tau=0.0, split_k=0, fast_restart=0, fast_eps=1e-3, muon=(0.0, 0.0, 0.0),
          spectral_init=0):
    abc = np.ascontiguousarray(np.asarray(abc, dtype=np.float64).reshape(-1))
    if abc.size != 3 * T:
        raise ValueError("abc must hold 3*T coefficients")
    pred = 0
    if predictor is not None:
        if predictor.numel() != MLP_PARAMS or not predictor.is_cuda or predictor.dtype != _torch().float32:
            raise ValueError("predictor must be a float32 device tensor of MLP_PARAMS values")
        pred = predictor.data_ptr()
    o = Opts(int(T), abc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), COMPUTE[compute],
             int(fp8_steps), int(norm_mode), int(tile), pred, int(force_class), float(fallback_tau),
             int(split_k), int(fast_restart), float(fast_eps), float(muon[0]), float(muon[1]),
             float(muon[2]), int(spectral_init))
    return o, abc


def _torch():
    import torch
    return torch


def _schedule(T, ell, abc):
    if abc is None:
        abc = coeffs(ell, T).abc
    return np.asarray(abc, dtype=np.float64).reshape(T, 3)


def _workspace(nbytes, device):
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    base = buf.data_ptr()
    off = (-base) % 256
    return buf, base + off


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def workspace_size(shapes, T=5, compute="bf16", fp8_steps=0) -> int:
    mats = (Matrix * max(1, len(shapes)))()
    for i, (m, n) in enumerate(shapes):
        mats[i] = Matrix(1, 1, m, n, n, n, PE_BF16, PE_BF16)
    o, _keep = _opts(T, np.zeros(3 * T), compute, fp8_steps, 0, 0)
    return int(lib().pe_workspace_size(len(shapes), mats, ctypes.byref(o)))


# ------------------------------------------------------------ l-predictor
def mlp_forward(params, feats, stream=None):
    """logits (B x 8) of the predictor MLP (device kernels)."""
    torch = _torch()
    B = feats.shape[0]
    logits = torch.empty((B, CLASSES), dtype=torch.float32, device=feats.device)
    _check(lib().pe_mlp_forward(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(feats.data_ptr()),
                                B, ctypes.c_void_p(logits.data_ptr()), _stream(stream)),
           "pe_mlp_forward")
    return logits


def _mlp_ws(B, device):
    n = int(lib().pe_mlp_workspace_size(B))
    return _workspace(n, device) + (n,)


def mlp_grad(params, feats, labels, stream=None):
    """(mean cross-entropy, gradient) on the device."""
    torch = _torch()
    B = feats.shape[0]
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feats.device)
    loss = torch.empty(1, dtype=torch.float32, device=feats.device)
    buf, ws, n = _mlp_ws(B, feats.device)
    _check(lib().pe_mlp_grad(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(feats.data_ptr()),
                             ctypes.c_void_p(labels.data_ptr()), B, ctypes.c_void_p(grad.data_ptr()),
                             ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(ws), n, _stream(stream)),
           "pe_mlp_grad")
    return loss, grad


def load_predictor(path=None, T: int = 5, device="cuda"):
    """The committed l-predictor (weights trained by train_predictor on the
    device kernels) as a device tensor, and its metadata."""
    import json
    import torch
    base = path or os.path.join(HERE, f"predictor_T{T}")
    theta = np.load(base + ".npy", allow_pickle=False)
    with open(base + ".json") as f:
        meta = json.load(f)
    if theta.shape != (MLP_PARAMS,) or theta.dtype != np.float32:
        raise ValueError("predictor file does not hold MLP_PARAMS float32 values")
    if meta.get("T") != T:
        raise ValueError(f"predictor trained for T={meta.get('T')}, asked for T={T}")
    return torch.from_numpy(theta).to(device), meta


class MLPTrainer:
    """Adam on the device: params, moments and the per-step workspace stay resident."""

    def __init__(self, params, B):
        torch = _torch()
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = 0
        self.B = B
        self.loss = torch.empty(1, dtype=torch.float32, device=params.device)
        self._buf, self._ws, self._n = _mlp_ws(B, params.device)

    def train_step(self, feats, labels, lr, stream=None):
        assert feats.shape[0] == self.B
        self.step += 1
        _check(lib().pe_mlp_train_step(ctypes.c_void_p(self.params.data_ptr()),
                                       ctypes.c_void_p(self.m.data_ptr()),
                                       ctypes.c_void_p(self.v.data_ptr()), self.step, float(lr),
                                       ctypes.c_void_p(feats.data_ptr()),
                                       ctypes.c_void_p(labels.data_ptr()), self.B,
                                       ctypes.c_void_p(self.loss.data_ptr()), ctypes.c_void_p(self._ws),
                                       self._n, _stream(stream)), "pe_mlp_train_step")
        return self.loss


def polar(G, T: int = 5, ell: float = 1e-3, abc=None, compute: str = "bf16", out=None,
          out_dtype=None, fp8_steps: int = 0, norm_mode: int = 0, tile: int = 0, stream=None,
          predictor=None, force_class: int = -1, fallback_tau: float = 0.0, split_k: int = 0,
          fast_restart: int = 0, fast_eps: float = 1e-3, spectral_init: int = 0):
    """X_T for one matrix (pe_polar).  Returns a new tensor unless ``out`` is given."""
    return polar_batched([G], T, ell, abc, compute, [out] if out is not None else None,
                         out_dtype, fp8_steps, norm_mode, tile, stream, predictor, force_class,
                         fallback_tau, split_k=split_k, fast_restart=fast_restart,
                         fast_eps=fast_eps, spectral_init=spectral_init, _single=True)[0]


def polar_batched(Gs, T: int = 5, ell: float = 1e-3, abc=None, compute: str = "bf16", outs=None,
                  out_dtype=None, fp8_steps: int = 0, norm_mode: int = 0, tile: int = 0,
                  stream=None, predictor=None, force_class: int = -1, fallback_tau: float = 0.0,
                  split_k: int = 0, fast_restart: int = 0, fast_eps: float = 1e-3,
                  moms=None, weights=None, muon=(0.0, 0.0, 0.0), spectral_init: int = 0,
                  _single: bool = False):
    """X_T for a list of matrices of any shapes (pe_polar_batched).  With
    ``moms`` / ``weights`` (lists of device tensors, entries may be None) the
    Muon step is fused in: M <- beta M + (1-beta) G before the iteration and
    W <- (1 - lr wd) W - lr X_T after it, muon = (beta, lr, wd); ``outs`` may
    then hold None entries (no X written)."""
    import torch
    Gs = list(Gs)
    n = len(Gs)
    moms = list(moms) if moms is not None else [None] * n
    weights = list(weights) if weights is not None else [None] * n
    if outs is None:
        outs = [torch.empty(G.shape, dtype=out_dtype or G.dtype, device=G.device) for G in Gs]
    sched = _schedule(T, ell, abc)
    o, _keep = _opts(T, sched, compute, fp8_steps, norm_mode, tile, predictor, force_class,
                     fallback_tau, split_k, fast_restart, fast_eps, muon, spectral_init)
    mats = (Matrix * max(1, n))()
    for i, (G, X, M, W) in enumerate(zip(Gs, outs, moms, weights)):
        mats[i] = _matrix(G, X, M, W)
    L = lib()
    nbytes = int(L.pe_workspace_size(len(Gs), mats, ctypes.byref(o)))
    if nbytes == 0 and len(Gs) > 0:
        _invalid(L, len(Gs), mats, o)
    dev = Gs[0].device if Gs else None
    ws_buf, ws = _workspace(nbytes, dev) if Gs else (None, 0)
    st = _stream(stream)
    if _single:
        rc = L.pe_polar(mats, ctypes.byref(o), ctypes.c_void_p(ws), nbytes, st)
        where = "pe_polar"
    else:
        rc = L.pe_polar_batched(len(Gs), mats, ctypes.byref(o), ctypes.c_void_p(ws), nbytes, st)
        where = "pe_polar_batched"
    _check(rc, where)
    if ws_buf is not None:
        # keep the workspace alive until the stream has consumed it
        ws_buf.record_stream(torch.cuda.current_stream() if stream is None else stream)
    return outs


NOALLOC_SCRATCH_BYTES = 128 << 20


def polar_noalloc(G, out, T: int = 5, ell: float = 1e-3, abc=None, compute: str = "bf16",
                  fp8_steps: int = 0, norm_mode: int = 0, tile: int = 0, split_k: int = 0,
                  stream=None):
    """X_T for one matrix into the caller's ``out`` with the library's static
    workspace (pe_polar_noalloc: no device allocation by the library or here)."""
    sched = _schedule(T, ell, abc)
    o, _keep = _opts(T, sched, compute, fp8_steps, norm_mode, tile, split_k=split_k)
    mat = _matrix(G, out)
    L = lib()
    _check(L.pe_polar_noalloc(ctypes.byref(mat), ctypes.byref(o), _stream(stream)),
           "pe_polar_noalloc")
    return out


def muon_step(Gs, moms, weights, lr: float, beta: float = 0.9, wd: float = 0.0, T: int = 5,
              ell: float = 1e-3, abc=None, compute: str = "bf16", outs=None, **kw):
    """One Muon optimizer step over a list of weight matrices (Section 1.1):
    M <- beta M + (1 - beta) G, W <- (1 - lr wd) W - lr polar(M), with
    polar(M) from Polar Express, all in grouped launches (pe_polar_batched).
    Updates ``moms`` (FP32) and ``weights`` in place; returns ``outs`` (None
    entries unless given)."""
    outs = list(outs) if outs is not None else [None] * len(list(Gs))
    return polar_batched(Gs, T, ell, abc, compute, outs, moms=moms, weights=weights,
                         muon=(beta, lr, wd), **kw)


def quantize_e4m3(x, scale: float, stream=None):
    """e4m3 bytes of x * scale with the FP8 path's device conversion."""
    import torch
    x = x.contiguous().view(-1)
    q = torch.empty(x.numel(), dtype=torch.uint8, device=x.device)
    _check(lib().pe_quantize_e4m3(ctypes.c_void_p(x.data_ptr()), _dtype_code(x.dtype),
                                  ctypes.c_void_p(q.data_ptr()), x.numel(), float(scale),
                                  _stream(stream)), "pe_quantize_e4m3")
    return q


class Plan:
    """Tile tables built once and the T-step sequence captured as a hipGraph."""

    def __init__(self, Gs, outs=None, T: int = 5, ell: float = 1e-3, abc=None, compute: str = "bf16",
                 out_dtype=None, fp8_steps: int = 0, norm_mode: int = 0, tile: int = 0, stream=None,
                 predictor=None, force_class: int = -1, fallback_tau: float = 0.0,
                 ws_fill=None, split_k: int = 0, fast_restart: int = 0, fast_eps: float = 1e-3,
                 moms=None, weights=None, muon=(0.0, 0.0, 0.0), spectral_init: int = 0):
        import torch
        self.Gs = list(Gs)
        n = len(self.Gs)
        self.moms = list(moms) if moms is not None else [None] * n
        self.weights = list(weights) if weights is not None else [None] * n
        self.outs = outs if outs is not None else [
            torch.empty(G.shape, dtype=out_dtype or G.dtype, device=G.device) for G in self.Gs]
        self.T = T
        self.abc = _schedule(T, ell, abc)
        self._predictor = predictor
        o, self._abc_keep = _opts(T, self.abc, compute, fp8_steps, norm_mode, tile, predictor,
                                  force_class, fallback_tau, split_k, fast_restart, fast_eps, muon,
                                  spectral_init)
        self._mats = (Matrix * max(1, n))()
        for i, (G, X, M, W) in enumerate(zip(self.Gs, self.outs, self.moms, self.weights)):
            self._mats[i] = _matrix(G, X, M, W)
        L = lib()
        self.ws_bytes = int(L.pe_workspace_size(len(self.Gs), self._mats, ctypes.byref(o)))
        if self.ws_bytes == 0:
            _invalid(L, len(self.Gs), self._mats, o)
        self._ws_buf, self._ws = _workspace(self.ws_bytes, self.Gs[0].device)
        if ws_fill is not None:
            # the library must not depend on the workspace's prior contents
            self._ws_buf.fill_(int(ws_fill) & 0xFF)
        h = ctypes.c_void_p()
        _check(L.pe_plan_create(len(self.Gs), self._mats, ctypes.byref(o), ctypes.c_void_p(self._ws),
                                self.ws_bytes, _stream(stream), ctypes.byref(h)), "pe_plan_create")
        self._h = h

    def launch(self, graph: bool = True, stream=None):
        _check(lib().pe_plan_launch(self._h, _stream(stream), 1 if graph else 0), "pe_plan_launch")
        return self.outs

    def selection(self, stream=None):
        """(classes, features, estimates, fallback flags) of a learned plan's last
        launch, read on ``stream`` (the launch's; default the current stream)."""
        n = len(self.Gs)
        cls = np.zeros(n, dtype=np.int32)
        flags = np.zeros(n, dtype=np.int32)
        feats = np.zeros((n, FEATURES), dtype=np.float32)
        est = np.zeros(n, dtype=np.float32)
        _check(lib().pe_plan_selection(self._h, _stream(stream), cls.ctypes.data, feats.ctypes.data,
                                       est.ctypes.data, flags.ctypes.data), "pe_plan_selection")
        return cls, feats, est, flags

    def launch_phase(self, step: int, phase: int, stream=None):
        """Diagnostic: one phase (0 norm, 1 Gram, 2 A^2+combine, 3 update) of one step."""
        _check(lib().pe_plan_launch_phase(self._h, int(step), int(phase), _stream(stream)),
               "pe_plan_launch_phase")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pe_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
