"""Oracle: storage formats, rounding and dequantisation of stored data.

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

Rounding is round-to-nearest, ties to even (Sec. 4.1 uses round-to-nearest),
written from its definition: a value a > 0 with leading bit 2^e is rounded
to a multiple of the quantum 2^(max(e, emin) - m), m = stored mantissa bits,
emin = smallest normal exponent; numpy's round() breaks ties to even.  The
unit roundoffs of Table 1 follow from m: u = 2^-(m+1).

Formats (code: mantissa bits, smallest normal exponent, largest finite):
  0 FP64  52  -1022  ~1.8e308
  1 FP32  23  -126   ~3.4e38
  2 BF16   7  -126   ~3.39e38
  3 FP16  10  -14    65504
  4 FP8 E4M3 (OCP, no infinities)  3  -6  448

Column scaling: the narrow-exponent formats FP16 and FP8 carry one scale per
column, c = max(fl32(max|col| / largest finite), 2^-126) (c = 1 for an
all-zero column), so the column's largest entry lands on the top of the
format's range; the stored code is q = sat(round(col / c)), saturated at the
largest finite value.  FP64, FP32 and BF16 (FP32's exponent range) use c = 1.  The dequantised entry c*q is exact in float64
(at most 11 significant bits times 24), so the stored matrix the product
must reach is known exactly.
"""
from __future__ import annotations

import numpy as np

F64, F32, BF16, F16, FP8 = 0, 1, 2, 3, 4
VALR = 5
NAMES = {F64: "f64", F32: "f32", BF16: "bf16", F16: "f16", FP8: "fp8e4m3"}
MANT = {F64: 52, F32: 23, BF16: 7, F16: 10, FP8: 3}
EMIN = {F64: -1022, F32: -126, BF16: -126, F16: -14, FP8: -6}
MAXF = {F64: np.finfo(np.float64).max,
        F32: float(np.finfo(np.float32).max),
        BF16: (2.0 - 2.0 ** -7) * 2.0 ** 127,
        F16: 65504.0,
        FP8: 448.0}
BYTES = {F64: 8, F32: 4, BF16: 2, F16: 2, FP8: 1}


def unit_roundoff(fmt: int) -> float:
    """u = 2^-(m+1) for m stored mantissa bits (Table 1)."""
    return 2.0 ** -(MANT[fmt] + 1)


def round_fmt(v: np.ndarray, fmt: int) -> np.ndarray:
    """Round float64 values to the nearest value of `fmt` (ties to even),
    saturating at the largest finite value.  Returns float64."""
    v = np.asarray(v, dtype=np.float64)
    if fmt == F64:
        return v.copy()
    a = np.abs(v)
    out = np.zeros_like(a)
    nz = a > 0
    _, E = np.frexp(a[nz])                 # a = f * 2^E, f in [0.5, 1)
    e = np.maximum(E - 1, EMIN[fmt])        # exponent of the leading bit
    quantum = np.ldexp(1.0, e - MANT[fmt])
    out[nz] = np.round(a[nz] / quantum) * quantum
    out = np.minimum(out, MAXF[fmt])
    return np.copysign(out, v)


def column_scales(A: np.ndarray, fmt: int) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    if fmt in (F64, F32, BF16) or A.shape[0] == 0:
        return np.ones(A.shape[1])
    m = np.abs(A).max(axis=0)
    c = (m / MAXF[fmt]).astype(np.float32).astype(np.float64)
    c = np.maximum(c, 2.0 ** -126)
    c[m == 0.0] = 1.0
    return c


def quantize_columns(A: np.ndarray, fmt: int):
    """(codes as float64, per-column scales) for a matrix stored in `fmt`."""
    A = np.asarray(A, dtype=np.float64)
    c = column_scales(A, fmt)
    Q = round_fmt(A / c[None, :], fmt) if A.size else A.copy()
    return Q, c


def dequantize_columns(Q: np.ndarray, c: np.ndarray) -> np.ndarray:
    return np.asarray(Q) * np.asarray(c)[None, :]


def stored(A: np.ndarray, fmt: int) -> np.ndarray:
    """The matrix as the product sees it after storing it in `fmt`."""
    if A is None:
        return None
    Q, c = quantize_columns(A, fmt)
    return np.asfortranarray(dequantize_columns(Q, c))
