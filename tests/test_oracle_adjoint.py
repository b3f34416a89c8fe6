"""Pins of the oracle's adjoint product (the remark after Alg. 3): the
transposed matrix expands to exactly the transpose of the dense expansion,
the adjoint identity <y, M x> = <M^T y, x> holds to rounding for every
format, the rank-1 kernel gives its closed form, and the stored adjoint
under a policy is the policy applied to the transposed blocks."""
import numpy as np
import pytest

from conftest import cached
from oracle import adjoint, mvm, stored, trees
from synth import (KERNEL_LAPLACE, KERNEL_RANK1, compress_h, gaussian_vector, rank1_factors, sphere_points,
                   to_h2, to_uh)


def case(kernel=KERNEL_LAPLACE, n=1200, kind="standard"):
    def build():
        p = sphere_points(n, 41)
        st = trees.build_structure(p, kind=kind)
        h = compress_h(p, kernel, st, 1e-8, method="svd")
        return p, st, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("adj", kernel, n, kind), build)


def expand(st, fmt, v):
    if fmt == "h":
        return mvm.h_to_dense(st, v.dense, v.W, v.sigma, v.X)
    if fmt == "uh":
        return mvm.uh_to_dense(st, v.dense, v.row_basis, v.col_basis, v.coupling)
    rb = mvm.h2_explicit_bases(st, v.row_leaf_basis, v.row_transfer)
    cb = mvm.h2_explicit_bases(st, v.col_leaf_basis, v.col_transfer)
    return mvm.uh_to_dense(st, v.dense, rb, cb, v.coupling)


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_expansion_is_the_transpose(fmt):
    p, st, vals = case()
    A = expand(st, fmt, vals[fmt])
    At = expand(adjoint.transpose_structure(st), fmt, adjoint.transpose_values(fmt, vals[fmt]))
    # the same factors multiplied in another order: equal up to rounding
    assert np.abs(At - A.T).max() <= 1e-14 * np.abs(A).max()
    dense_b = [b for b in range(st.nblocks) if not st.blk_adm[b]]
    tv = adjoint.transpose_values(fmt, vals[fmt])
    assert all(np.array_equal(tv.dense[b], vals[fmt].dense[b].T) for b in dense_b)


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("kind", ["standard", "hodlr"])
def test_adjoint_identity(fmt, kind):
    p, st, vals = case(kind=kind, n=900)
    n = st.n
    x, y = gaussian_vector(n, 1), gaussian_vector(n, 2)
    Ax = stored.product(st, fmt, vals[fmt], 1.0, x, np.zeros(n))
    Aty = adjoint.product(st, fmt, vals[fmt], 1.0, y, np.zeros(n))
    assert abs(y @ Ax - Aty @ x) <= 1e-13 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_rank1_closed_form():
    """k(x, y) = f(x) g(y) with a zero diagonal: (A^T x)_j = g_j (f . x) - f_j g_j x_j."""
    p, st, vals = case(kernel=KERNEL_RANK1, n=700)
    f, g = rank1_factors(p)
    x, y0 = gaussian_vector(st.n, 3), gaussian_vector(st.n, 4)
    want = y0 - 0.5 * (g * (f @ x) - f * g * x)
    for fmt in ("h", "uh", "h2"):
        out = adjoint.product(st, fmt, vals[fmt], -0.5, x, y0)
        assert np.linalg.norm(out - want) <= 1e-12 * np.linalg.norm(want - y0), fmt


def test_stored_adjoint_applies_the_policy_to_the_transposed_blocks():
    """FP32 storage rounds every entry on its own (no scales), so storing
    the transposed blocks gives exactly the transposes of the stored blocks."""
    p, st, vals = case()
    tst = adjoint.transpose_structure(st)
    for fmt in ("h", "uh", "h2"):
        sv = stored.stored_values(st, fmt, vals[fmt], dense="f32", factor="f32", eps=1e-6)
        tv = stored.stored_values(tst, fmt, adjoint.transpose_values(fmt, vals[fmt]), dense="f32", factor="f32",
                                  eps=1e-6)
        want = adjoint.transpose_values(fmt, sv)
        for name in ("dense", "coupling", "W", "X", "row_basis", "col_basis", "row_leaf_basis", "col_leaf_basis",
                     "row_transfer", "col_transfer"):
            a, b = getattr(tv, name, None), getattr(want, name, None)
            if a is None:
                continue
            assert all((u is None and w is None) or np.array_equal(u, w) for u, w in zip(a, b)), (fmt, name)
