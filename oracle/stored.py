"""Oracle: the matrix as stored under a precision policy.

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

Direct compression (Sec. 4.1) of every stored matrix, column by column, with
the per-column scale rule of oracle.quant.  The policy follows the storage
classes of the paper: dense inadmissible blocks (diagonal blocks t == s may
use their own format), low-rank factors / cluster bases (Sec. 4.2), and
coupling and transfer matrices (direct compression, Sec. 4.1).  For the H^2
column transfers F the scaled axis is a row of F.  The result is a copy of
the values with every stored matrix replaced by its dequantised version, so
the products in oracle.mvm give the exact product of the stored matrix.
"""
from __future__ import annotations

import copy

import numpy as np

from . import quant

DT = {"f64": quant.F64, "f32": quant.F32, "bf16": quant.BF16, "f16": quant.F16, "fp8": quant.FP8}


def _s(A, fmt):
    return None if A is None else quant.stored(A, DT[fmt])


def _s_rows(A, fmt):
    return None if A is None else np.asfortranarray(quant.stored(np.asarray(A).T, DT[fmt]).T)


def stored_values(st, fmt: str, values, dense="f64", diag=None, factor="f64", coupling=None):
    diag = diag or dense
    coupling = coupling or factor
    out = copy.copy(values)
    out.dense = [None if values.dense[b] is None else
                 _s(values.dense[b], diag if st.blk_tau[b] == st.blk_sigma[b] else dense)
                 for b in range(st.nblocks)]
    if fmt == "h":
        out.W = [_s(a, factor) for a in values.W]
        out.X = [_s(a, factor) for a in values.X]
    elif fmt == "uh":
        out.row_basis = [_s(a, factor) for a in values.row_basis]
        out.col_basis = [_s(a, factor) for a in values.col_basis]
        out.coupling = [_s(a, coupling) for a in values.coupling]
    else:
        out.row_leaf_basis = [_s(a, factor) for a in values.row_leaf_basis]
        out.col_leaf_basis = [_s(a, factor) for a in values.col_leaf_basis]
        out.row_transfer = [_s(a, coupling) for a in values.row_transfer]
        out.col_transfer = [_s_rows(a, coupling) for a in values.col_transfer]
        out.coupling = [_s(a, coupling) for a in values.coupling]
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
