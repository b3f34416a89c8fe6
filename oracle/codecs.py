"""Oracle: the byte-aligned floating-point codecs of Sec. 4.1, FPX and AFLP.

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

FPX (the table of custom formats in Sec. 4.1): a value is kept as the
leading bytes of its FP32 (e = 8 exponent bits) or FP64 (e = 11) encoding,
with m stored mantissa bits, 1 + e + m a multiple of 8, rounded to nearest
(ties to even).  Exponent range, bias and subnormals are those of FP32 /
FP64; values beyond the largest finite value saturate.  Rows:
    (e, m) = (8, 7) (8, 15) (8, 23) (11, 28) (11, 36) (11, 44) (11, 52)
the (8, 7) row is the BF16 layout, (8, 23) FP32 and (11, 52) FP64.  For an
accuracy eps the row is the first whose m is at least
m_eps = ceil(-log2 eps) (the printed table assigns m = 7 to m_eps up to 10,
which would not meet eps for m_eps = 8..10; the first row with m >= m_eps
is taken instead).

AFLP (Sec. 4.1): per stored column a sign bit, e exponent bits and m'
mantissa bits, 1 + e + m' = 8B for B bytes.  The reading implemented here
(the paper fixes the bit budget and the idea of scaling so the exponent
field holds only the data's dynamic range, not the exact encoding):
  - the column is scaled by a power of two c = 2^k, k = floor(log2 vmin),
    vmin the smallest nonzero magnitude, so every nonzero |v|/c >= 1;
  - a nonzero value |v|/c = 2^E (1 + f), E >= 0, is stored with exponent
    code z = E + 1 and the m' bits of f rounded to nearest (ties to even;
    a carry moves to the next exponent); z = 0 with zero mantissa is the
    exact zero; a value above the largest code saturates to it;
  - the decoded value is sign * c * 2^(z-1) * (1 + M / 2^m'), exact in
    float64 for every m' <= 52;
  - e (one per stored matrix: a dense block, a coupling or transfer matrix,
    a low-rank factor or cluster basis) is the fewest bits holding the
    largest code z = floor(log2(vmax/c)) + 1 of any of its columns.  With
    the zero code and the power-of-two scale this is the paper's
    e_dr = ceil(log2 log2(vmax/vmin)) or at most two bits more.
  - direct compression at accuracy eps takes B = ceil((1 + e + m_eps) / 8)
    and m' = 8B - 1 - e >= m_eps (the mantissa widened to fill the bytes).
The storage widths are B = 1 .. 7; 1 + e + m' > 56 is FP64.  Widths up to
3 bytes decode through float32 and need e <= 7; wider ones decode through
float64 and need e <= 10 (beyond: the next width, else FP64).
"""
from __future__ import annotations

import math

import numpy as np

from . import quant

# storage codes of the codec formats (the numbering of the C interface)
FPX24, FPX40, FPX48, FPX56 = 6, 7, 8, 9
AFLP = {1: 10, 2: 11, 3: 12, 4: 13, 5: 14, 6: 15, 7: 16}   # bytes -> code
AFLP_WIDTH = {v: k for k, v in AFLP.items()}
AFLP_AUTO, FPX_AUTO = 17, 18

FPX_ROWS = ((8, 7), (8, 15), (8, 23), (11, 28), (11, 36), (11, 44), (11, 52))
FPX_CODE = {(8, 7): quant.BF16, (8, 15): FPX24, (8, 23): quant.F32, (11, 28): FPX40,
            (11, 36): FPX48, (11, 44): FPX56, (11, 52): quant.F64}
FPX_SHAPE = {v: k for k, v in FPX_CODE.items()}
FPX_LADDER = tuple(FPX_CODE[r] for r in FPX_ROWS)

NAMES = {FPX24: "fpx24", FPX40: "fpx40", FPX48: "fpx48", FPX56: "fpx56",
         **{c: f"aflp{8 * b}" for b, c in AFLP.items()}}


def is_fpx(code: int) -> bool:
    return code in (FPX24, FPX40, FPX48, FPX56)


def is_aflp(code: int) -> bool:
    return code in AFLP_WIDTH


def nbytes(code: int) -> int:
    """Bytes of one stored value (the nominal width, before tiling)."""
    if is_aflp(code):
        return AFLP_WIDTH[code]
    if is_fpx(code):
        e, m = FPX_SHAPE[code]
        return (1 + e + m) // 8
    return quant.BYTES[code]


def m_eps(eps: float) -> int:
    """m_eps = ceil(-log2 eps) (Sec. 4.1), at least 0, evaluated exactly:
    with eps = g 2^E, g in [0.5, 1), -log2 eps = -E - log2 g and
    -log2 g lies in (0, 1], so the ceiling is 1 - E."""
    _, E = math.frexp(eps)
    return max(0, 1 - E)


# ---------------------------------------------------------------- FPX

def fpx_round(v, e: int, m: int) -> np.ndarray:
    """Round float64 values to the FPX format (e, m): round to nearest, ties
    to even, subnormals below 2^emin, saturation at the largest finite
    value.  emin = 2 - 2^(e-1), emax = 2^(e-1) - 1."""
    v = np.asarray(v, dtype=np.float64)
    if (e, m) == (11, 52):
        return v.copy()
    emin = 2 - 2 ** (e - 1)
    emax = 2 ** (e - 1) - 1
    maxf = math.ldexp(2.0 - 2.0 ** -m, emax)
    a = np.abs(v)
    out = np.zeros_like(a)
    nz = a > 0
    _, E = np.frexp(a[nz])                   # a = f 2^E, f in [0.5, 1)
    lead = np.maximum(E - 1, emin)           # exponent of the leading bit
    quantum = np.ldexp(1.0, lead - m)
    out[nz] = np.round(a[nz] / quantum) * quantum
    out = np.minimum(out, maxf)
    return np.copysign(out, v)


def fpx_row(eps: float):
    """The FPX row for accuracy eps: first row with m >= m_eps (None:
    FP64, eps below 2^-52)."""
    need = m_eps(eps)
    for e, m in FPX_ROWS:
        if m >= need:
            return (e, m)
    return None


def fpx_code_for_eps(eps: float) -> int:
    r = fpx_row(eps)
    return quant.F64 if r is None else FPX_CODE[r]


def fpx_stored(A, code: int) -> np.ndarray:
    """A stored in FPX format `code` (a BF16/FP32/FP64 code means the
    matching row)."""
    e, m = FPX_SHAPE[code]
    return fpx_round(A, e, m)


def fpx_bits(q: float, code: int) -> int:
    """The B-byte FPX code of an already rounded value: the leading bytes
    of its FP32 (e = 8) or FP64 (e = 11) encoding."""
    e, m = FPX_SHAPE[code]
    B = (1 + e + m) // 8
    if e == 8:
        w = int(np.array([q], dtype=np.float32).view(np.uint32)[0])
        return w >> (32 - 8 * B)
    w = int(np.array([q], dtype=np.float64).view(np.uint64)[0])
    return w >> (64 - 8 * B)


# ---------------------------------------------------------------- AFLP
# Every function works on whole matrices, column by column (numpy along
# axis 0); a 1-D argument is one column.

def _cols(A) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    return A[:, None] if A.ndim == 1 else A


def aflp_scale_exps(A) -> np.ndarray:
    """k of every column's scale c = 2^k: floor(log2 vmin) over the nonzero
    magnitudes (0 for an all-zero column)."""
    a = np.abs(_cols(A))
    vmin = np.where(a > 0, a, np.inf).min(axis=0, initial=np.inf)
    k = np.zeros(a.shape[1], dtype=np.int64)
    ok = np.isfinite(vmin)
    _, E = np.frexp(vmin[ok])                    # vmin = g 2^E, g in [0.5, 1)
    k[ok] = E - 1
    return k


def aflp_scale_exp(col) -> int:
    return int(aflp_scale_exps(col)[0])


def aflp_column_ebits_all(A) -> np.ndarray:
    """Fewest exponent bits of every column: bit length of its largest code
    z = floor(log2(vmax / c)) + 1 (at least 1)."""
    a = np.abs(_cols(A))
    vmax = a.max(axis=0, initial=0.0)
    _, zmax = np.frexp(np.ldexp(vmax, -aflp_scale_exps(A)))   # vmax/c = f 2^z, f in [0.5, 1)
    _, bits = np.frexp(zmax.astype(np.float64))                # bit length of z (0 for z = 0)
    return np.maximum(bits, 1)


def aflp_column_ebits(col) -> int:
    return int(aflp_column_ebits_all(col)[0])


def aflp_ebits(A) -> int:
    """e of a stored matrix: the largest column requirement."""
    A = _cols(A)
    if A.shape[1] == 0:
        return 1
    return int(aflp_column_ebits_all(A).max())


def aflp_feasible(B: int, e: int) -> bool:
    """Width B holds exponent width e: a nonnegative mantissa, and the
    exponent fits the float32 (B <= 3, e <= 7) or float64 (e <= 10) decode."""
    if not 1 <= B <= 7 or 8 * B - 1 - e < 0:
        return False
    return e <= (7 if B <= 3 else 10)


def aflp_encode(A, e: int, B: int):
    """Codes (sign, z, M) of every entry and the scale exponent k of every
    column."""
    A = _cols(A)
    mp = 8 * B - 1 - e
    k = aflp_scale_exps(A)
    a = np.ldexp(np.abs(A), -k[None, :])         # exact: power-of-two scales
    nz = a > 0
    sign = (np.signbit(A) & nz).astype(np.int64)
    z = np.zeros(A.shape, dtype=np.int64)
    M = np.zeros(A.shape, dtype=np.int64)
    f, E = np.frexp(a[nz])                       # a = f 2^E, f in [0.5, 1)
    E = E.astype(np.int64) - 1                   # a = 2^E (1 + frac)
    frac = 2.0 * f - 1.0                         # exact
    Mi = np.round(np.ldexp(frac, mp)).astype(np.int64)   # exact scaling; ties to even
    carry = Mi == (1 << mp)
    Mi[carry] = 0
    E[carry] += 1
    zi = E + 1
    sat = zi > (1 << e) - 1                      # saturate at the largest code
    zi[sat] = (1 << e) - 1
    Mi[sat] = (1 << mp) - 1
    z[nz] = zi
    M[nz] = Mi
    return sign, z, M, k


def aflp_decode_all(sign, z, M, k, e: int, B: int) -> np.ndarray:
    """sign * 2^k * 2^(z-1) * (1 + M / 2^m') entry by entry (k per column);
    z = 0 is zero."""
    mp = 8 * B - 1 - e
    z = np.asarray(z, dtype=np.int64)
    kk = np.asarray(k, dtype=np.int64)
    mag = np.ldexp(1.0 + np.ldexp(np.asarray(M, dtype=np.float64), -mp), z - 1 + (kk[None, :] if z.ndim == 2 else kk))
    mag[z == 0] = 0.0
    return np.where(np.asarray(sign) != 0, -mag, mag)


def aflp_encode_column(col, e: int, B: int):
    """Codes (sign, z, M) of one column and its scale exponent k."""
    s, z, M, k = aflp_encode(col, e, B)
    return s[:, 0], z[:, 0], M[:, 0], int(k[0])


def aflp_decode(sign, z, M, k: int, e: int, B: int) -> np.ndarray:
    return aflp_decode_all(sign, z, M, k, e, B)


def aflp_code_word(s: int, z: int, M: int, e: int, B: int) -> int:
    """The B-byte code: sign | z (e bits) | M (m' bits), most significant first."""
    mp = 8 * B - 1 - e
    return (s << (8 * B - 1)) | (z << mp) | M


def aflp_stored(A, e: int, B: int) -> np.ndarray:
    """Every column of A stored in AFLP width B with exponent width e."""
    s_, z, M, k = aflp_encode(A, e, B)
    return np.asfortranarray(aflp_decode_all(s_, z, M, k, e, B))


def aflp_stored_column(col, e: int, B: int) -> np.ndarray:
    return aflp_stored(col, e, B)[:, 0]


def aflp_direct_width(e: int, eps: float):
    """Direct compression (Sec. 4.1): B = ceil((1 + e + m_eps) / 8), moved
    to the next feasible width; None = FP64."""
    B = max(1, -(-(1 + e + m_eps(eps)) // 8))
    while B <= 7 and not aflp_feasible(B, e):
        B += 1
    return B if B <= 7 else None


# ---------------------------------------------------------------- selection

def column_error2(w, s) -> float:
    """Squared 2-norm of w - s, squares summed in row order."""
    return float(column_errors2(w, s)[0])


def column_errors2(A, S) -> np.ndarray:
    """Squared 2-norms of the columns of A - S, squares summed in row order."""
    d = _cols(A) - _cols(S)
    if d.shape[0] == 0:
        return np.zeros(d.shape[1])
    return np.cumsum(d * d, axis=0)[-1]


def valr_aflp_widths(A, deltas, e: int):
    """VALR (Sec. 4.2) with AFLP: column j takes the narrowest feasible
    width whose stored column differs from it by at most deltas[j] in the
    2-norm (None: FP64)."""
    A = _cols(A)
    d2 = np.asarray(deltas, dtype=np.float64) ** 2
    out = [None] * A.shape[1]
    for B in range(7, 0, -1):                    # narrower widths overwrite wider ones
        if not aflp_feasible(B, e):
            continue
        ok = column_errors2(A, aflp_stored(A, e, B)) <= d2
        for j in np.flatnonzero(ok):
            out[j] = B
    return out


def valr_fpx_codes(A, deltas):
    """VALR with FPX: column j takes the first row of the table whose stored
    column meets its budget (the last row is FP64)."""
    A = _cols(A)
    d2 = np.asarray(deltas, dtype=np.float64) ** 2
    out = [quant.F64] * A.shape[1]
    for code in reversed(FPX_LADDER[:-1]):       # earlier rows overwrite later ones
        ok = column_errors2(A, fpx_stored(A, code)) <= d2
        for j in np.flatnonzero(ok):
            out[j] = code
    return out
