"""Round-to-nearest-even low-precision formats, written from their definitions
(test infrastructure, see package doc).

* bfloat16: the upper 16 bits of an IEEE binary32 after rounding the discarded
  16 bits to nearest, ties to even (8 exponent bits, 7 stored mantissa bits).
* OCP FP8 E4M3 ("e4m3fn"): 1 sign, 4 exponent (bias 7), 3 mantissa bits; no
  infinities; the largest finite magnitude is 448 = 1.75 * 2^8; subnormals
  m/8 * 2^-6; here values beyond 448 saturate to +-448 (the per-tensor scale of
  the FP8 variant maps the largest magnitude to 448).

Both are computed in float64 from the value, so they serve as independent
statements of what the device conversions must produce.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def round_bf16(x) -> np.ndarray:
    """float32 -> bfloat16 (RNE) -> float64 values."""
    x = np.asarray(x, dtype=np.float32)
    out = np.empty(x.shape, dtype=np.float64)
    xf = x.astype(np.float64)
    finite = np.isfinite(xf)
    ax = np.abs(xf)
    # exponent of the leading bit for normal binary32 values
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.maximum(e, -126.0)            # bf16 subnormals share binary32's
    ulp = np.ldexp(1.0, (e - 7).astype(np.int64))
    q = np.round(xf / ulp) * ulp         # np.round is half-to-even
    out[:] = np.where(finite, q, xf)
    out[ax == 0] = xf[ax == 0]
    return out


def round_e4m3(x, saturate: bool = True) -> np.ndarray:
    """float64 -> OCP E4M3 (RNE, saturating) -> float64 values."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.maximum(e, -6.0)              # below 2^-6 the spacing is fixed: subnormals
    ulp = np.ldexp(1.0, (e - 3).astype(np.int64))
    q = np.round(ax / ulp) * ulp
    if saturate:
        q = np.minimum(q, E4M3_MAX)
    q = np.where(ax == 0, 0.0, q)
    return np.copysign(q, x)


def e4m3_code(x) -> np.ndarray:
    """Bit pattern (uint8) of round_e4m3(x): s eeee mmm."""
    q = round_e4m3(x)
    sign = (np.signbit(q)).astype(np.uint16) << 7
    a = np.abs(q)
    code = np.zeros(q.shape, dtype=np.uint16)
    sub = (a > 0) & (a < 2.0 ** -6)
    code[sub] = np.round(a[sub] / 2.0 ** -9).astype(np.uint16)
    nrm = a >= 2.0 ** -6
    e = np.floor(np.log2(np.where(nrm, a, 1.0)))
    m = np.round((a / np.ldexp(1.0, e.astype(np.int64)) - 1.0) * 8.0)
    code[nrm] = (((e[nrm] + 7).astype(np.uint16) << 3) | m[nrm].astype(np.uint16))
    return (code | sign).astype(np.uint8)


def iteration_bf16_operands(G, abc):
    """Model of the bf16 path's rounding points, in float64 otherwise.

    The scale sigma = 1/(1.01 ||G||_F + 1e-7) multiplies step 1's products
    after rounding, so step 1 takes the operand bf16(G) and
        A_1 = sigma^2 bf16(G) bf16(G)^T,  X_1 = sigma (a G + bf16(B_1) bf16(G));
    later steps take bf16(X) for the Gram product and the update, bf16(A) for
    A^2 and for the b A term of B, and bf16(B) for the update, while the a X
    term uses the unrounded iterate (the FP32 master).  The distance of this model from the FP64
    iteration is the part of the error that bf16 operands cause at all; it sets
    a per-input tolerance where the 3e-2 bar is out of reach of the arithmetic."""
    G = np.asarray(G, dtype=np.float64)
    m, n = G.shape
    tall = m > n
    Gt = G.T if tall else G
    sigma = 1.0 / (1.01 * np.sqrt(np.sum(G * G)) + 1e-7)
    X = Gt.copy()
    for t, (a, b, c) in enumerate(np.asarray(abc, dtype=np.float64).reshape(-1, 3)):
        scale = sigma if t == 0 else 1.0
        Xo = round_bf16(X.astype(np.float32))
        A = scale * scale * (Xo @ Xo.T)
        Ao = round_bf16(A.astype(np.float32))
        B = b * Ao + c * (Ao @ Ao)
        X = scale * (a * X + round_bf16(B.astype(np.float32)) @ Xo)
    return X.T if tall else X
