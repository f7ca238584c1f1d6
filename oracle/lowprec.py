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
