"""Pins of the oracle's codecs (FPX and AFLP, Sec. 4.1) and of the codec
storage policies (Sec. 4.1-4.2), against values derived by hand, the FPX
table as printed, integer rounding of IEEE bit patterns, and the error
bounds the formats guarantee."""
import math
import pathlib

import numpy as np
import pytest

from oracle import codecs, quant, stored

GOLD = pathlib.Path(__file__).parent / "golden"


def _hex_f64(h):
    return float(np.array([int(h, 16)], dtype=np.uint64).view(np.float64)[0])


def _golden():
    fpx, aflp = [], []
    for line in (GOLD / "codec_examples.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        kind, rest = line.split(maxsplit=1)
        if kind == "fpx":
            name, x, code, val = rest.split()
            fpx.append((stored.DT[name], _hex_f64(x), int(code, 16), _hex_f64(val)))
        else:
            head, ke, codes, vals = [p.strip() for p in rest.split("|")]
            B, xs = head.split()
            k, e = ke.split()
            aflp.append((int(B), [float(v) for v in xs.split(",")], int(k), int(e),
                         [int(c, 16) for c in codes.split(",")], [float(v) for v in vals.split(",")]))
    return fpx, aflp


def test_fpx_worked_examples():
    fpx, _ = _golden()
    assert len(fpx) == 8
    for code, x, want_code, want in fpx:
        q = float(codecs.fpx_stored(np.array([x]), code)[0])
        assert q == want, (code, x)
        assert codecs.fpx_bits(q, code) == want_code, (code, x)


def test_aflp_worked_examples():
    _, aflp = _golden()
    assert len(aflp) == 3
    for B, xs, k, e, codes, vals in aflp:
        col = np.array(xs)
        assert codecs.aflp_scale_exp(col) == k
        assert codecs.aflp_ebits(col[:, None]) == e
        s, z, M, kk = codecs.aflp_encode_column(col, e, B)
        assert kk == k
        words = [codecs.aflp_code_word(int(a), int(b), int(c), e, B) for a, b, c in zip(s, z, M)]
        assert words == codes, (B, xs)
        assert list(codecs.aflp_decode(s, z, M, k, e, B)) == vals


def test_fpx_table_rows_as_printed():
    """The selection reproduces every row of the printed table (lo..hi of
    ceil(-log2 eps) -> (e, m)), except m_eps = 8..10 of the first row, where
    the first row that meets the accuracy is taken."""
    rows = []
    for line in (GOLD / "fpx_table.txt").read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            rows.append(tuple(int(v) for v in line.split()))
    assert [(e, m) for _, _, e, m in rows] == list(codecs.FPX_ROWS)
    for lo, hi, e, m in rows:
        for need in range(lo, hi + 1):
            eps = 2.0 ** -need
            assert codecs.m_eps(eps) == need
            got = codecs.fpx_row(eps)
            if need <= m:
                assert got == (e, m), need
            else:
                assert got == (8, 15) and lo == 0, need
    assert codecs.fpx_row(2.0 ** -53) is None


def test_m_eps_is_the_exact_ceiling():
    assert codecs.m_eps(1e-6) == 20 and codecs.m_eps(1e-8) == 27 and codecs.m_eps(1e-4) == 14
    assert codecs.m_eps(2.0 ** -20) == 20
    assert codecs.m_eps(2.0 ** -20 * (1 - 2.0 ** -53)) == 21       # just below a power of two
    assert codecs.m_eps(2.0 ** -20 * (1 + 2.0 ** -52)) == 20
    assert codecs.m_eps(0.75) == 1 and codecs.m_eps(1.0) == 0 and codecs.m_eps(4.0) == 0


def _rne_bits(bits: int, drop: int) -> int:
    """Round an unsigned bit pattern to `drop` fewer bits, ties to even
    (integer arithmetic on the IEEE encoding; valid away from overflow)."""
    lsb = (bits >> drop) & 1
    return (bits + (1 << (drop - 1)) - 1 + lsb) >> drop


def test_fpx_matches_integer_rounding_of_ieee_patterns():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(4000) * np.exp(rng.uniform(-20, 20, 4000))
    x32 = x.astype(np.float32).astype(np.float64)       # exactly representable in FP32
    # (8, 23): FP32 itself, both by numpy's conversion and the oracle
    assert np.array_equal(codecs.fpx_round(x, 8, 23), x.astype(np.float32).astype(np.float64))
    # (8, 7) and (8, 15) of FP32-representable values: RNE of the FP32 pattern
    for m in (7, 15):
        got = codecs.fpx_round(x32, 8, m)
        drop = 23 - m
        for xi, gi in zip(x32, got):
            b = int(np.array([abs(xi)], dtype=np.float32).view(np.uint32)[0])
            r = _rne_bits(b, drop) << drop
            want = float(np.array([r], dtype=np.uint32).view(np.float32)[0])
            assert abs(gi) == want and math.copysign(1, gi) == math.copysign(1, xi)
    # (11, m): RNE of the FP64 pattern
    for m in (28, 36, 44):
        got = codecs.fpx_round(x, 11, m)
        drop = 52 - m
        for xi, gi in zip(x[:500], got[:500]):
            b = int(np.array([abs(xi)], dtype=np.float64).view(np.uint64)[0])
            r = _rne_bits(b, drop) << drop
            assert abs(gi) == float(np.array([r], dtype=np.uint64).view(np.float64)[0])
    assert np.array_equal(codecs.fpx_round(x, 11, 52), x)
    # FPX (8, 7) is the BF16 storage of the hardware ladder
    assert np.array_equal(codecs.fpx_round(x, 8, 7), quant.round_fmt(x, quant.BF16))


def test_fpx_bits_are_the_leading_bytes():
    rng = np.random.default_rng(12)
    for code in (codecs.FPX24, codecs.FPX40, codecs.FPX48, codecs.FPX56):
        e, m = codecs.FPX_SHAPE[code]
        B = (1 + e + m) // 8
        q = codecs.fpx_stored(rng.standard_normal(50), code)
        for v in q:
            c = codecs.fpx_bits(float(v), code)
            assert c < (1 << (8 * B))
            if e == 8:
                back = float(np.array([c << (32 - 8 * B)], dtype=np.uint32).view(np.float32)[0])
            else:
                back = float(np.array([c << (64 - 8 * B)], dtype=np.uint64).view(np.float64)[0])
            assert back == v


def test_aflp_round_trip_bounds_and_invariants():
    rng = np.random.default_rng(13)
    for trial in range(60):
        m = int(rng.integers(1, 200))
        col = rng.standard_normal(m) * np.exp(rng.uniform(-8, 8, m) * (trial % 3))
        col[rng.random(m) < 0.05] = 0.0
        e = codecs.aflp_ebits(col[:, None])
        for B in range(1, 8):
            if not codecs.aflp_feasible(B, e):
                continue
            mp = 8 * B - 1 - e
            assert 1 + e + mp == 8 * B
            s, z, M, k = codecs.aflp_encode_column(col, e, B)
            q = codecs.aflp_decode(s, z, M, k, e, B)
            assert np.all((z >= 0) & (z < (1 << e)) & (M >= 0) & (M < (1 << mp)))
            assert np.array_equal(q == 0, col == 0)                 # zero exact, only zero
            assert np.all(np.signbit(q[col != 0]) == np.signbit(col[col != 0]))
            sat = (z == (1 << e) - 1) & (M == (1 << mp) - 1)
            rel = np.abs(q - col)[col != 0] / np.abs(col[col != 0])
            ok = ~sat[col != 0]
            assert np.all(rel[ok] <= 2.0 ** -(mp + 1))             # round to nearest
            assert np.all(rel <= 2.0 ** -mp)                       # saturation within one step
            # a power-of-two rescaling of the column rescales the stored column
            q2 = codecs.aflp_stored_column(col * 2.0 ** 7, e, B)
            assert np.array_equal(q2, q * 2.0 ** 7)


def test_aflp_exponent_width_against_the_paper_formula():
    """e is the paper's e_dr = ceil(log2 log2(vmax/vmin)) or at most two
    bits more (zero code, power-of-two scale), and never less than what the
    codes need."""
    rng = np.random.default_rng(14)
    for _ in range(300):
        r = 2.0 ** rng.uniform(1.1, 60)
        col = np.concatenate([[1.0, r], rng.uniform(1.0, r, 10)]) * 2.0 ** rng.uniform(-30, 30)
        e = codecs.aflp_ebits(col[:, None])
        a = np.abs(col)
        edr = math.ceil(math.log2(math.log2(a.max() / a.min())))
        assert edr <= e <= edr + 2
        _, z, _, _ = codecs.aflp_encode_column(col, e, 7)
        assert z.max() < (1 << e)


def test_aflp_direct_width_from_eps():
    for e in range(1, 11):
        for need in range(0, 56):
            B = codecs.aflp_direct_width(e, 2.0 ** -need)
            if B is None:
                assert 1 + e + need > 56 - 0 or e > 10
                continue
            assert codecs.aflp_feasible(B, e)
            assert 8 * B - 1 - e >= need
            assert B == max(1, -(-(1 + e + need) // 8)) or not codecs.aflp_feasible(B - 1, e)


def test_codec_valr_columns_meet_budgets_minimally():
    """VALR with either codec: each column's stored error is within its
    budget, and the next narrower choice would miss it."""
    rng = np.random.default_rng(15)
    A = np.linalg.qr(rng.standard_normal((80, 12)))[0]
    sigma = np.logspace(0, -9, 12)
    deltas = stored.h_block_deltas(sigma, 1e-6)
    e = codecs.aflp_ebits(A)
    widths = codecs.valr_aflp_widths(A, deltas, e)
    for j, B in enumerate(widths):
        w = A[:, j]
        if B is not None:
            assert codecs.column_error2(w, codecs.aflp_stored_column(w, e, B)) <= deltas[j] ** 2
        lower = (B or 8) - 1
        while lower >= 1 and not codecs.aflp_feasible(lower, e):
            lower -= 1
        if lower >= 1:
            assert codecs.column_error2(w, codecs.aflp_stored_column(w, e, lower)) > deltas[j] ** 2
    assert len(set(widths)) > 2                      # the budgets spread over several widths
    fcodes = codecs.valr_fpx_codes(A, deltas)
    for j, c in enumerate(fcodes):
        w = A[:, j]
        assert codecs.column_error2(w, codecs.fpx_stored(w, c)) <= deltas[j] ** 2
        i = codecs.FPX_LADDER.index(c)
        if i > 0:
            assert codecs.column_error2(w, codecs.fpx_stored(w, codecs.FPX_LADDER[i - 1])) > deltas[j] ** 2


@pytest.mark.parametrize("policy", ["aflp", "fpx"])
@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_codec_policies_meet_the_accuracy(policy, fmt):
    """The stored matrix under the codec policies stays within the VALR
    bounds: its product differs from the unstored product by O(eps)
    (Fig. 8: the compressed formats follow eps), and every stored entry
    is counted once."""
    from synth import KERNEL_LAPLACE, compress_h, gaussian_vector, sphere_points, to_h2, to_uh
    from oracle import trees
    p = sphere_points(1024, 77)
    st = trees.build_structure(p)
    h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
    vals = {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}[fmt]
    x, y = gaussian_vector(st.n, 5), gaussian_vector(st.n, 6)
    exact = stored.product(st, fmt, vals, 1.0, x, y)
    for eps in (1e-4, 1e-6, 1e-8):
        counts = np.zeros(stored.NCODES, dtype=np.int64)
        sv = stored.stored_values(st, fmt, vals, dense=policy, diag=policy, factor=policy, eps=eps, counts=counts)
        got = stored.product(st, fmt, sv, 1.0, x, y)
        err = np.linalg.norm(got - exact) / np.linalg.norm(exact - y)
        assert err <= 20 * eps, (eps, err)
        sv64 = stored.stored_values(st, fmt, vals, eps=eps)
        total = sum(a.size for a in vars(sv64).values() if isinstance(a, list) for a in a
                    if isinstance(a, np.ndarray) and a.ndim == 2)
        assert counts.sum() == total
        used = {c for c in range(stored.NCODES) if counts[c]}
        fam = set(codecs.AFLP.values()) if policy == "aflp" else set(codecs.FPX_LADDER)
        assert used <= fam | {quant.F64}, used
