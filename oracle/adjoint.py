"""Oracle: the adjoint product y := alpha * M^T * x + y.

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

The remark after Alg. 3 computes M^H x over block columns; all data is
real, so M^H = M^T.  M^T is again a hierarchical matrix of the same form over
the same cluster tree: its leaf blocks are the transposes of M's, block
(tau, sigma) of M becoming (sigma, tau).  Per block:
  dense    D^T;
  H        (W diag(s) X^T)^T = X diag(s) W^T, so W and X swap;
  UH       (W_t S X_s^T)^T = X_s S^T W_t^T, so the row and column cluster
           bases (ranks, weights) swap and the coupling is transposed;
  H^2      as UH, and the row and column transfer matrices swap.
The adjoint product is then the ordinary product of that matrix.
"""
from __future__ import annotations

import copy

import numpy as np

from synth.inputs import Structure


def transpose_structure(st: Structure) -> Structure:
    """The same cluster tree with every block (tau, sigma) as (sigma, tau)."""
    t = Structure(st.n, st.perm, st.begin, st.end, st.level, st.parent, st.son0, st.son1,
                  np.array(st.blk_sigma), np.array(st.blk_tau), np.array(st.blk_adm))
    for k in ("bbox", "partition"):
        if k in st._cache:
            t._cache[k] = st._cache[k]
    return t


def _tr(a):
    return None if a is None else np.asfortranarray(np.asarray(a).T)


def transpose_values(fmt: str, values):
    """The value set of M^T (same container type, blocks indexed as in M)."""
    v = copy.copy(values)
    v.dense = [_tr(a) for a in values.dense]
    if fmt == "h":
        v.W, v.X = values.X, values.W
        return v
    v.row_sv, v.col_sv = values.col_sv, values.row_sv
    v.coupling = [_tr(a) for a in values.coupling]
    if fmt == "uh":
        v.row_basis, v.col_basis = values.col_basis, values.row_basis
    else:
        v.row_rank, v.col_rank = values.col_rank, values.row_rank
        v.row_leaf_basis, v.col_leaf_basis = values.col_leaf_basis, values.row_leaf_basis
        v.row_transfer, v.col_transfer = values.col_transfer, values.row_transfer
    return v


def product(st: Structure, fmt: str, values, alpha, x, y):
    """y + alpha * M^T x for the (already stored) values of M."""
    from . import stored
    return stored.product(transpose_structure(st), fmt, transpose_values(fmt, values), alpha, x, y)
