"""Pins of the oracle's VALR storage (Sec. 4.2) and of its direct
compression rule (Sec. 4.1 with Table 1), against facts fixed outside the
oracle: independent float32 / float16 / bfloat16 roundings written here
from the IEEE definitions, the error bounds of eq. (6) and eq. (7), and
special columns whose stored error is known exactly."""
import numpy as np
import pytest

from conftest import cached
from oracle import quant, stored, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_vector, sphere_points, to_h2, to_uh


# --- roundings written from the IEEE definitions, independent of oracle.quant
def via_float32(w):
    return w.astype(np.float32).astype(np.float64)


def via_float16(w):
    """Column scale as the storage rule defines it, then an IEEE binary16
    round trip (numpy's float16 conversion is round-to-nearest-even)."""
    m = np.abs(w).max() if len(w) else 0.0
    c = 1.0 if m == 0.0 else max(float(np.float32(m / 65504.0)), 2.0 ** -126)
    return (w / c).astype(np.float16).astype(np.float64) * c


def via_bfloat16(w):
    """bfloat16 = the top 16 bits of float32, rounded to nearest even on the
    dropped 16 bits (w is first rounded to float32: exact for these tests,
    whose inputs are float32 values or far from the bf16 rounding points)."""
    u = w.astype(np.float32).view(np.uint32).astype(np.uint64)
    lower = u & 0xFFFF
    top = u >> 16
    up = (lower > 0x8000) | ((lower == 0x8000) & ((top & 1) == 1))
    top = (top + up.astype(np.uint64)) & 0xFFFF
    return (top << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def err2(w, s):
    d = w - s
    return float(np.cumsum(d * d)[-1]) if len(d) else 0.0


def test_direct_format_follows_table1():
    # cheapest format whose unit roundoff (Table 1) is at most eps
    assert stored.direct_format(0.1) == quant.FP8        # u = 2^-4
    assert stored.direct_format(2.0 ** -4) == quant.FP8
    assert stored.direct_format(1e-3) == quant.F16       # u = 2^-11 (2 bytes, finer than BF16)
    assert stored.direct_format(1e-4) == quant.F32
    assert stored.direct_format(1e-6) == quant.F32       # u = 2^-24
    assert stored.direct_format(2.0 ** -24) == quant.F32
    assert stored.direct_format(1e-8) == quant.F64
    assert stored.direct_format(1e-16) == quant.F64


def test_valr_choice_is_feasible_and_cheapest():
    """The chosen format meets the budget and every cheaper candidate misses
    it, checked with roundings independent of the oracle's (FP8 has no
    independent numpy type; its rounding is pinned exhaustively elsewhere)."""
    rng = np.random.default_rng(7)
    indep = {quant.F32: via_float32, quant.F16: via_float16, quant.BF16: via_bfloat16,
             quant.FP8: lambda w: quant.stored(w[:, None], quant.FP8)[:, 0]}
    order = [quant.FP8, quant.F16, quant.BF16, quant.F32, quant.F64]
    seen = set()
    for trial in range(400):
        m = int(rng.integers(1, 90))
        w = rng.standard_normal(m).astype(np.float32).astype(np.float64)   # exact in float32
        w /= 2.0 ** int(rng.integers(-3, 4))                              # still exact
        nrm = np.linalg.norm(w)
        delta = nrm * 10.0 ** rng.uniform(-9, -0.5)
        f = stored.valr_column_format(w, delta)
        seen.add(f)
        if f != quant.F64:
            assert err2(w, indep[f](w)) <= delta * delta
        for g in order[:order.index(f)]:
            assert err2(w, indep[g](w)) > delta * delta, (trial, f, g)
    # float32-exact columns never need FP64; every cheaper level is reached
    assert quant.F64 not in seen
    assert {quant.FP8, quant.F16, quant.F32} <= seen


def test_valr_special_columns():
    z = np.zeros(17)
    assert stored.valr_column_format(z, 0.0) == quant.FP8          # zero column: exact in any format
    assert stored.valr_column_format(np.zeros(0), 0.0) == quant.FP8
    w = np.array([1.0, -0.5, 0.25, 448.0, 3.0 * 2.0 ** -6])        # exact FP8 E4M3 values (scale 1)
    assert stored.valr_column_format(w, 0.0) == quant.FP8
    rng = np.random.default_rng(3)
    g = rng.standard_normal(50)
    assert stored.valr_column_format(g, 0.0) == quant.F64          # generic float64 data
    assert stored.valr_column_format(g, np.inf) == quant.FP8       # unlimited budget
    g32 = g.astype(np.float32).astype(np.float64)
    assert stored.valr_column_format(g32, 0.0) == quant.F32
    # budget just below / at the FP16 error of the column
    e16 = np.sqrt(err2(g32, via_float16(g32)))
    e8 = np.sqrt(err2(g32, quant.stored(g32[:, None], quant.FP8)[:, 0]))
    assert e16 < e8
    assert stored.valr_column_format(g32, e16) == quant.F16
    assert stored.valr_column_format(g32, np.nextafter(e16, 0.0)) != quant.F16


def test_valr_budgets():
    s = np.array([4.0, 3.0, 0.0])
    d = stored.h_block_deltas(s, 1e-6)
    assert d[0] == pytest.approx(1e-6 * 5.0 / 7.0 / 4.0)            # ||s|| = 5, 1 + 2k = 7
    assert d[1] == pytest.approx(1e-6 * 5.0 / 7.0 / 3.0)
    assert d[2] == np.inf
    b = stored.basis_deltas(np.array([4.0, 3.0]), 1e-6)
    assert b[0] == pytest.approx(1e-6 * 5.0 / 2.0 / 4.0)            # delta = eps ||sv|| / k
    assert len(stored.basis_deltas(np.zeros(0), 1e-6)) == 0


def _h(eps):
    def build():
        p = sphere_points(2048, 1001)
        st = trees.build_structure(p)
        h = compress_h(p, KERNEL_LAPLACE, st, eps, method="svd")
        return st, h, to_uh(h, st), to_h2(h, st)
    return cached(("valr-oracle", eps), build)


@pytest.mark.slow
@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_eq6_bound_per_h_block(eps):
    """eq. (6): with delta_i = delta / sigma_i and delta = eps ||sigma|| / (1+2k)
    the stored block W~ S X~^T stays within eps ||sigma||_F of W S X^T."""
    st, h, _, _ = _h(eps)
    sv = stored.stored_values(st, "h", h, factor="valr", dense="f64", eps=eps)
    worst = 0.0
    nblk = 0
    for b in np.nonzero(st.blk_adm)[0]:
        s = h.sigma[b]
        if s is None or len(s) == 0:
            continue
        A = (h.W[b] * s) @ h.X[b].T
        B = (sv.W[b] * s) @ sv.X[b].T
        r = np.linalg.norm(A - B) / (eps * np.linalg.norm(s))
        worst = max(worst, r)
        nblk += 1
    assert nblk > 100
    assert worst <= 1.0, worst


@pytest.mark.slow
def test_eq6_bound_fails_without_compensation(monkeypatch):
    """A planted mistake in the oracle (delta = eps ||sigma||, the 1 + 2k
    compensation dropped) must break the eq. (6) check above."""
    eps = 1e-6
    st, h, _, _ = _h(eps)
    budgets = stored.valr_deltas
    monkeypatch.setattr(stored, "h_block_deltas",
                        lambda s, e: budgets(s, e * np.linalg.norm(np.asarray(s, dtype=np.float64))))
    sv = stored.stored_values(st, "h", h, factor="valr", dense="f64", eps=eps)
    worst = 0.0
    for b in np.nonzero(st.blk_adm)[0]:
        s = h.sigma[b]
        if s is None or len(s) == 0:
            continue
        A = (h.W[b] * s) @ h.X[b].T
        B = (sv.W[b] * s) @ sv.X[b].T
        worst = max(worst, np.linalg.norm(A - B) / (eps * np.linalg.norm(s)))
    assert worst > 1.0


@pytest.mark.slow
@pytest.mark.parametrize("fmt", ["uh", "h2"])
def test_eq7_bound_per_basis(fmt):
    """eq. (7): ||(W - W~) Sigma||_F <= k delta = eps ||Sigma||_F for every
    (leaf) basis stored under VALR."""
    eps = 1e-6
    st, h, uh, h2 = _h(eps)
    vals = uh if fmt == "uh" else h2
    sv = stored.stored_values(st, fmt, vals, factor="valr", dense="f64", coupling="f64", eps=eps)
    pairs = ((vals.row_basis, sv.row_basis, vals.row_sv), (vals.col_basis, sv.col_basis, vals.col_sv)) \
        if fmt == "uh" else ((vals.row_leaf_basis, sv.row_leaf_basis, vals.row_sv),
                             (vals.col_leaf_basis, sv.col_leaf_basis, vals.col_sv))
    nb = 0
    for orig, st_b, svs in pairs:
        for A, B, s in zip(orig, st_b, svs):
            if A is None or A.shape[1] == 0:
                continue
            assert np.linalg.norm((A - B) * s[None, :]) <= eps * np.linalg.norm(s)
            nb += 1
    assert nb > 20


@pytest.mark.slow
@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_valr_product_error_and_savings(fmt, eps):
    """The product of the VALR-stored matrix stays within a small multiple
    of eps of the float64 product of the same factors, and every stored entry
    is counted once (the stored bytes, tile padding included, are compared
    with uniform FP32 on the library's plan in test_abi_host)."""
    st, h, uh, h2 = _h(eps)
    vals = {"h": h, "uh": uh, "h2": h2}[fmt]
    n = st.n
    x = gaussian_vector(n, 21)
    y0 = np.zeros(n)
    ref = stored.product(st, fmt, vals, 1.0, x, y0)
    counts = np.zeros(6, dtype=np.int64)
    sv = stored.stored_values(st, fmt, vals, dense="valr", diag="valr", factor="valr", eps=eps, counts=counts)
    out = stored.product(st, fmt, sv, 1.0, x, y0)
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    assert err <= 3.0 * eps, err
    diag = sum(h.dense[b].size for b in range(st.nblocks)
               if h.dense[b] is not None and st.blk_tau[b] == st.blk_sigma[b])
    assert counts[quant.F64] >= diag                     # diagonal near field stays FP64
    # Sec. 4.2/4.3: VALR stores fewer bytes than uniform FP32 storage with
    # the same FP64 diagonal near field (counted on the stored entries)
    stored_b = sum(int(counts[f]) * quant.BYTES[f] for f in range(5))
    total = int(counts[:5].sum())
    assert stored_b < 4 * (total - diag) + 8 * diag, (stored_b, total, diag)
    assert counts[:5].sum() == sum(a.size for a in vals.dense if a is not None) + sum(
        a.size for grp in ((vals.W, vals.X) if fmt == "h" else
                           (vals.row_basis, vals.col_basis, vals.coupling) if fmt == "uh" else
                           (vals.row_leaf_basis, vals.col_leaf_basis, vals.row_transfer, vals.col_transfer,
                            vals.coupling))
        for a in grp if a is not None)


def test_factor_formats_are_per_column():
    """Sec. 4.2 decides every column on its own budget: the format of a
    column does not depend on its neighbours.  Two FP8-exact columns next to
    five columns that need FP16 stay FP8, and the choice of every column of a
    factor equals the choice for that column alone."""
    rng = np.random.default_rng(11)
    m = 40
    A = rng.standard_normal((m, 7))
    exact8 = quant.stored(A, quant.FP8)                   # columns exactly FP8-representable
    base = np.column_stack([A[:, :5], exact8[:, 5:]])
    loose16 = [np.sqrt(err2(base[:, j], via_float16(base[:, j]))) * 1.0000001 for j in range(5)]
    deltas = loose16 + [0.0, 0.0]                         # FP16 for 0..4, FP8 (exact) for 5, 6
    assert stored.valr_factor_formats(base, deltas) == [quant.F16] * 5 + [quant.FP8] * 2
    B = rng.standard_normal((m, 12))
    d = list(np.geomspace(1e-1, 1e-9, 12))
    whole = stored.valr_factor_formats(B, d)
    alone = [stored.valr_factor_formats(B[:, j:j + 1], [d[j]])[0] for j in range(12)]
    assert whole == alone
    assert len(set(whole)) >= 3                           # the budgets span several formats
