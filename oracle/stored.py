"""Oracle: the matrix as stored under a precision policy.

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

Direct compression (Sec. 4.1) of every stored matrix, column by column, with
the per-column scale rule of oracle.quant.  The policy follows the storage
classes of the paper: dense inadmissible blocks (diagonal blocks t == s may
use their own format), low-rank factors / cluster bases (Sec. 4.2), and
coupling and transfer matrices (direct compression, Sec. 4.1).  For the H^2
column transfers F the scaled axis is a row of F.  Under VALR (Sec. 4.2)
each column of a low-rank factor or cluster basis gets the cheapest format
that meets its own error budget, and the other classes the cheapest format
whose unit roundoff is at most eps.  The policies "aflp" and "fpx" do the
same with the paper's own codecs (oracle.codecs): direct compression of the
dense, coupling and transfer classes at eps, VALR over the codec's widths
for factors and bases (one AFLP exponent width per stored matrix).  Fixed
codec widths ("fpx24", "aflp24", ...) store a class in that format.  The
result is a copy of
the values with every stored matrix replaced by its dequantised version, so
the products in oracle.mvm give the exact product of the stored matrix.
"""
from __future__ import annotations

import copy

import numpy as np

from . import codecs, quant

DT = {"f64": quant.F64, "f32": quant.F32, "bf16": quant.BF16, "f16": quant.F16, "fp8": quant.FP8,
      "valr": quant.VALR, "aflp": codecs.AFLP_AUTO, "fpx": codecs.FPX_AUTO,
      **{name: code for code, name in codecs.NAMES.items()}}
ADAPTIVE = (quant.VALR, codecs.AFLP_AUTO, codecs.FPX_AUTO)
NCODES = 19


def direct_format(eps: float) -> int:
    """Direct compression (Sec. 4.1) under VALR: the cheapest format (fewest
    bytes, then smallest unit roundoff) whose unit roundoff (Table 1) is at
    most eps; FP64 if none is."""
    for f in sorted((quant.FP8, quant.F16, quant.BF16, quant.F32),
                    key=lambda f: (quant.BYTES[f], quant.unit_roundoff(f))):
        if quant.unit_roundoff(f) <= eps:
            return f
    return quant.F64


def valr_column_format(w: np.ndarray, delta: float) -> int:
    """VALR (Sec. 4.2): the cheapest format whose stored column differs from
    w by at most delta in the 2-norm, trying FP8, FP16, BF16, FP32 in that
    order (FP64 otherwise).  The squared error is summed in row order and
    compared with delta^2."""
    w = np.asarray(w, dtype=np.float64)
    for f in (quant.FP8, quant.F16, quant.BF16, quant.F32):
        d = w - quant.stored(w[:, None], f)[:, 0]
        e2 = np.cumsum(d * d)[-1] if len(d) else 0.0
        if e2 <= delta * delta:
            return f
    return quant.F64


def valr_factor_formats(A, deltas) -> list:
    """VALR formats of the columns of one factor (Sec. 4.2): column j is
    stored in the cheapest format whose error meets its own budget
    deltas[j], independently of every other column."""
    A = np.asarray(A, dtype=np.float64)
    return [valr_column_format(A[:, j], deltas[j]) for j in range(A.shape[1])]


def _norm2(s) -> float:
    s = np.asarray(s, dtype=np.float64)
    return float(np.sqrt(np.cumsum(s * s)[-1])) if len(s) else 0.0


def valr_deltas(weights, delta: float) -> np.ndarray:
    """Per-column budgets delta_i = delta / weight_i (Sec. 4.2); a column of
    zero weight contributes nothing and gets an unlimited budget."""
    w = np.asarray(weights, dtype=np.float64)
    out = np.full(len(w), np.inf)
    nz = w > 0
    out[nz] = delta / w[nz]
    return out


def h_block_deltas(sigma, eps: float) -> np.ndarray:
    """Budgets of the columns of W_b and X_b of an H block with singular
    values sigma: delta = eps ||sigma||_2 / (1 + 2k), so the bound of eq. (6)
    on the stored block is the truncation error eps ||sigma||_2."""
    k = len(sigma)
    return valr_deltas(sigma, eps * _norm2(sigma) / (1.0 + 2.0 * k))


def basis_deltas(sv, eps: float) -> np.ndarray:
    """Budgets of the columns of a cluster basis with weights sv (the
    singular values of its construction): delta = eps ||sv||_2 / k, eq. (7)."""
    k = len(sv)
    return valr_deltas(sv, eps * _norm2(sv) / k) if k else np.zeros(0)


class _Store:
    """Stores matrices under one policy and counts the entries per format."""

    def __init__(self, eps, counts):
        self.eps = eps
        self.counts = counts

    def _count(self, f, entries):
        if self.counts is not None:
            self.counts[f] += entries

    def direct(self, A, fmt):
        if A is None:
            return None
        f = DT[fmt]
        A = np.asarray(A, dtype=np.float64)
        if f == quant.VALR:
            f = direct_format(self.eps)
        elif f == codecs.FPX_AUTO:
            f = codecs.fpx_code_for_eps(self.eps)
        elif f == codecs.AFLP_AUTO or codecs.is_aflp(f):
            return self._aflp_direct(A, f)
        self._count(f, A.size)
        if codecs.is_fpx(f):
            return np.asfortranarray(codecs.fpx_stored(A, f))
        return quant.stored(A, f)

    def _aflp_direct(self, A, f):
        """AFLP over a whole stored matrix: one exponent width e; the width
        from eps (policy) or at least the requested one (fixed)."""
        if A.size == 0:
            return A.copy()
        e = codecs.aflp_ebits(A)
        if f == codecs.AFLP_AUTO:
            B = codecs.aflp_direct_width(e, self.eps)
        else:
            B = codecs.AFLP_WIDTH[f]
            while B <= 7 and not codecs.aflp_feasible(B, e):
                B += 1
            B = B if B <= 7 else None
        if B is None:
            self._count(quant.F64, A.size)
            return np.asfortranarray(A.copy())
        self._count(codecs.AFLP[B], A.size)
        return codecs.aflp_stored(A, e, B)

    def direct_rows(self, A, fmt):
        """Direct compression with the scaled axis along the rows of A."""
        if A is None:
            return None
        return np.asfortranarray(self.direct(np.asarray(A).T, fmt).T)

    def factor(self, A, fmt, deltas):
        """A low-rank factor or cluster basis: one format for all columns,
        or under VALR one format per column chosen from its budget."""
        if A is None:
            return None
        f = DT[fmt]
        if f not in ADAPTIVE:
            return self.direct(A, fmt)
        A = np.asarray(A, dtype=np.float64)
        out = np.zeros_like(A, order="F")
        if f == quant.VALR:
            for j, fj in enumerate(valr_factor_formats(A, deltas)):
                self._count(fj, A.shape[0])
                out[:, j] = quant.stored(A[:, j:j + 1], fj)[:, 0]
        elif f == codecs.FPX_AUTO:
            codes = codecs.valr_fpx_codes(A, deltas)
            for fj in sorted(set(codes)):
                cols = [j for j, c in enumerate(codes) if c == fj]
                self._count(fj, A.shape[0] * len(cols))
                out[:, cols] = codecs.fpx_stored(A[:, cols], fj)
        else:
            e = codecs.aflp_ebits(A)                  # one exponent width per factor
            widths = codecs.valr_aflp_widths(A, deltas, e)
            for B in sorted(set(widths), key=lambda b: 8 if b is None else b):
                cols = [j for j, b in enumerate(widths) if b == B]
                if B is None:
                    self._count(quant.F64, A.shape[0] * len(cols))
                    out[:, cols] = A[:, cols]
                else:
                    self._count(codecs.AFLP[B], A.shape[0] * len(cols))
                    out[:, cols] = codecs.aflp_stored(A[:, cols], e, B)
        return out


def stored_values(st, fmt: str, values, dense="f64", diag=None, factor="f64", coupling=None,
                  eps: float = 0.0, counts=None):
    """The values as stored.  `counts` (length >= 19, optional) accumulates
    the stored entries per format code.  Under "valr" the dense and
    coupling/transfer classes are direct-compressed at eps, the diagonal
    dense blocks stay FP64, and factors/bases take VALR per column, which
    needs the singular values (H: sigma; UH/H2: row_sv/col_sv).  Under
    "aflp" / "fpx" every class given that policy, the diagonal blocks
    included, is compressed with the codec (Sec. 4.1-4.2)."""
    diag = diag or dense
    coupling = coupling or factor
    if DT[diag] == quant.VALR:
        diag = "f64"
    if any(DT[c] in ADAPTIVE for c in (dense, diag, factor, coupling)) and not eps > 0:
        raise ValueError("adaptive storage needs eps > 0")
    S = _Store(eps, counts)
    valr = DT[factor] in ADAPTIVE
    out = copy.copy(values)
    out.dense = [None if values.dense[b] is None else
                 S.direct(values.dense[b], diag if st.blk_tau[b] == st.blk_sigma[b] else dense)
                 for b in range(st.nblocks)]
    if fmt == "h":
        dl = [None if s is None else (h_block_deltas(s, eps) if valr else None) for s in values.sigma]
        out.W = [S.factor(a, factor, d) for a, d in zip(values.W, dl)]
        out.X = [S.factor(a, factor, d) for a, d in zip(values.X, dl)]
    elif fmt == "uh":
        def bd(sv):
            return [None if s is None else (basis_deltas(s, eps) if valr else None) for s in sv]
        rd = bd(values.row_sv) if valr else [None] * len(values.row_basis)
        cd = bd(values.col_sv) if valr else [None] * len(values.col_basis)
        out.row_basis = [S.factor(a, factor, d) for a, d in zip(values.row_basis, rd)]
        out.col_basis = [S.factor(a, factor, d) for a, d in zip(values.col_basis, cd)]
        out.coupling = [S.direct(a, coupling) for a in values.coupling]
    else:
        def bd(basis, sv):
            return [None if a is None else (basis_deltas(s, eps) if valr else None) for a, s in zip(basis, sv)]
        rd = bd(values.row_leaf_basis, values.row_sv) if valr else [None] * len(values.row_leaf_basis)
        cd = bd(values.col_leaf_basis, values.col_sv) if valr else [None] * len(values.col_leaf_basis)
        out.row_leaf_basis = [S.factor(a, factor, d) for a, d in zip(values.row_leaf_basis, rd)]
        out.col_leaf_basis = [S.factor(a, factor, d) for a, d in zip(values.col_leaf_basis, cd)]
        out.row_transfer = [S.direct(a, coupling) for a in values.row_transfer]
        out.col_transfer = [S.direct_rows(a, coupling) for a in values.col_transfer]
        out.coupling = [S.direct(a, coupling) for a in values.coupling]
    return out


def product(st, fmt: str, values, alpha, x, y):
    """y + alpha*M*x for already-stored values of any format (original order)."""
    from . import mvm
    if fmt == "h":
        return mvm.h_mvm(st, values.dense, values.W, values.sigma, values.X, alpha, x, y)
    if fmt == "uh":
        return mvm.uh_mvm(st, values.dense, values.row_basis, values.col_basis, values.coupling, alpha, x, y)
    return mvm.h2_mvm(st, values.dense, values.row_rank, values.col_rank, values.row_leaf_basis,
                      values.row_transfer, values.col_leaf_basis, values.col_transfer, values.coupling,
                      alpha, x, y)


def product_many(st, fmt: str, values, alpha, X, Y):
    """Many right-hand sides: column j of the result is the single-vector
    product (eq. 4) applied to column j of X and Y."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = np.empty_like(Y)
    for j in range(X.shape[1]):
        out[:, j] = product(st, fmt, values, alpha, X[:, j], Y[:, j])
    return out
