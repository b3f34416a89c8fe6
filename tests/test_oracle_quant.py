"""Pins for the oracle's storage formats (Table 1, Sec. 4.1 round-to-nearest).

Every code of BF16, FP16 and FP8 (E4M3) is decoded from its bit fields and
must be a fixed point of the rounding; midpoints must go to the even code;
the worst relative error in the normal range must equal the unit roundoff
printed in Table 1; FP32/FP16 rounding must agree with numpy's own casts."""
import os

import numpy as np
import pytest

from oracle import quant

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def decode_all(fmt):
    """All finite values of a format, decoded from the bit fields."""
    if fmt == quant.BF16:
        nbits, ebits, mbits, bias = 16, 8, 7, 127
    elif fmt == quant.F16:
        nbits, ebits, mbits, bias = 16, 5, 10, 15
    else:
        nbits, ebits, mbits, bias = 8, 4, 3, 7
    vals, codes = [], []
    for c in range(1 << nbits):
        s = c >> (nbits - 1)
        e = (c >> mbits) & ((1 << ebits) - 1)
        m = c & ((1 << mbits) - 1)
        if fmt == quant.FP8:
            if e == 15 and m == 7:
                continue                   # the only NaN encoding, no infinities
        elif e == (1 << ebits) - 1:
            continue                       # inf / nan
        if e == 0:
            v = m * 2.0 ** (1 - bias - mbits)
        else:
            v = (1.0 + m / 2.0 ** mbits) * 2.0 ** (e - bias)
        vals.append(-v if s else v)
        codes.append(c)
    return np.array(vals), np.array(codes)


@pytest.mark.parametrize("fmt", [quant.BF16, quant.F16, quant.FP8])
def test_every_code_is_a_fixed_point(fmt):
    v, _ = decode_all(fmt)
    assert np.array_equal(quant.round_fmt(v, fmt), v)
    assert np.abs(v).max() == quant.MAXF[fmt]


@pytest.mark.parametrize("fmt", [quant.BF16, quant.F16, quant.FP8])
def test_midpoints_round_to_even(fmt):
    v, codes = decode_all(fmt)
    pos = np.unique(v[v >= 0])
    mids = 0.5 * (pos[:-1] + pos[1:])
    r = quant.round_fmt(mids, fmt)
    # the code with an even last mantissa bit wins the tie
    lo_even = np.array([(c & 1) == 0 for c in
                        [codes[np.nonzero(v == a)[0][0]] for a in pos[:-1]]])
    expect = np.where(lo_even, pos[:-1], pos[1:])
    assert np.array_equal(r, expect)
    # just off the midpoint goes to the nearer neighbour
    up = np.nextafter(mids, np.inf)
    assert np.array_equal(quant.round_fmt(up, fmt), pos[1:])
    dn = np.nextafter(mids, -np.inf)
    assert np.array_equal(quant.round_fmt(dn, fmt), pos[:-1])


def test_unit_roundoff_matches_table1():
    printed = {}
    with open(os.path.join(GOLD, "table1_unit_roundoff.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, val = line.split()
                printed[name] = float(val)
    ours = {"FP64": quant.unit_roundoff(quant.F64), "FP32": quant.unit_roundoff(quant.F32),
            "BF16": quant.unit_roundoff(quant.BF16), "FP16": quant.unit_roundoff(quant.F16),
            "FP8": quant.unit_roundoff(quant.FP8), "TF32": 2.0 ** -11}
    for k, v in printed.items():
        assert float(f"{ours[k]:.2e}") == v, k


@pytest.mark.parametrize("fmt", [quant.F32, quant.BF16, quant.F16, quant.FP8])
def test_worst_relative_error_is_unit_roundoff(fmt):
    rng = np.random.default_rng(fmt)
    lo_norm = 2.0 ** quant.EMIN[fmt]
    hi = min(quant.MAXF[fmt], 1e30)
    a = np.exp(rng.uniform(np.log(lo_norm), np.log(hi), 200000))
    r = quant.round_fmt(a, fmt)
    relerr = np.abs(r - a) / a
    u = quant.unit_roundoff(fmt)
    assert relerr.max() <= u
    # the supremum u/(1+u) is approached just above a power of two
    assert relerr.max() > 0.99 * u / (1 + u)


def test_agrees_with_numpy_casts():
    rng = np.random.default_rng(3)
    v = rng.standard_normal(100000) * np.exp(rng.uniform(-30, 30, 100000))
    assert np.array_equal(quant.round_fmt(v, quant.F32), v.astype(np.float32).astype(np.float64))
    w = rng.standard_normal(100000) * np.exp(rng.uniform(-20, 10, 100000))
    assert np.array_equal(quant.round_fmt(w, quant.F16), w.astype(np.float16).astype(np.float64))


def test_saturation_and_column_scaling():
    assert quant.round_fmt(np.array([1e6, -500.0]), quant.FP8).tolist() == [448.0, -448.0]
    rng = np.random.default_rng(5)
    A = rng.standard_normal((50, 6))
    A[:, 2] = 0.0
    for fmt in (quant.BF16, quant.F16, quant.FP8):
        Q, c = quant.quantize_columns(A, fmt)
        assert np.array_equal(c.astype(np.float32).astype(np.float64), c)
        assert c[2] == 1.0 and not Q[:, 2].any()
        assert np.abs(Q).max() <= quant.MAXF[fmt]
        assert np.array_equal(quant.round_fmt(Q, fmt), Q)           # codes are representable
        D = quant.dequantize_columns(Q, c)
        # dequantisation is exact: dividing back recovers the codes
        assert np.array_equal(D / c[None, :], Q)
        u = quant.unit_roundoff(fmt)
        err = np.abs(D - A).max(axis=0)
        # near the top of the range the error is u relative; small entries
        # may fall below the normal range of the format (FP8 has 4 bits of
        # exponent range below its maximum)
        top = np.abs(A).max(axis=0)
        assert (err <= u * top * 1.0000001 + c * 2.0 ** (quant.EMIN[fmt] - quant.MANT[fmt])).all()
