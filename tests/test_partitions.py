"""BLR and HODLR partitions (the remark after Def. 2.3): the oracle's trees
pinned against their definitions, the library's layouts equal to the
oracle's bit for bit, and H / UH / H^2 products on them within the
truncation bound of the dense product."""
import numpy as np
import pytest

import paper_2405_03456_amd as hm
from conftest import cached
from oracle import dense, mvm, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_vector, sphere_points, to_h2, to_uh


def test_balanced_bisection_on_a_line():
    """Points on a line, leaf size 2: depth d = 3 for 7 points; every split
    takes the lower half (rounded down) along x; leaves hold 0 ... 1 ... 2
    points in x order."""
    xs = np.array([5.0, 1.0, 3.0, 7.0, 2.0, 6.0, 4.0])
    p = np.column_stack([xs, np.zeros(7), np.zeros(7)])
    st = trees.build_structure(p, leaf_size=2, kind=trees.HODLR)
    assert trees.balanced_depth(7, 2) == 2          # ceil(7/4) = 2 <= 2
    assert list(xs[st.perm]) == sorted(xs)
    leaves = [v for v in range(st.nnodes) if st.son0[v] < 0]
    assert [int(st.end[v] - st.begin[v]) for v in leaves] == [1, 2, 2, 2]
    assert all(st.level[v] == 2 for v in leaves)


@pytest.mark.parametrize("n", [1, 2, 65, 700, 2048])
def test_hodlr_structure(n):
    p = sphere_points(n, 31)
    st = trees.build_structure(p, kind=trees.HODLR)
    trees.validate_partition(st)
    inner = [v for v in range(st.nnodes) if st.son0[v] >= 0]
    leaves = [v for v in range(st.nnodes) if st.son0[v] < 0]
    adm = st.blk_adm.astype(bool)
    # every inner node contributes its two off-diagonal son blocks, every leaf its diagonal block
    assert adm.sum() == 2 * len(inner) and (~adm).sum() == len(leaves)
    for b in np.nonzero(adm)[0]:
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        assert t != s and st.parent[t] == st.parent[s]
    for b in np.nonzero(~adm)[0]:
        assert st.blk_tau[b] == st.blk_sigma[b] and st.son0[st.blk_tau[b]] < 0
    if n <= 2048:
        assert np.all(trees.coverage_bitmap(st) == 1)


@pytest.mark.parametrize("n", [1, 65, 700, 2048])
def test_blr_structure(n):
    p = sphere_points(n, 32)
    st = trees.build_structure(p, kind=trees.BLR)
    trees.validate_partition(st)
    leaves = [v for v in range(st.nnodes) if st.son0[v] < 0]
    assert st.nblocks == len(leaves) ** 2             # one level: every pair of leaves
    assert all(st.son0[t] < 0 and st.son0[s] < 0 for t, s in zip(st.blk_tau, st.blk_sigma))
    sizes = [int(st.end[v] - st.begin[v]) for v in leaves]
    assert max(sizes) - min(sizes) <= 1 and max(sizes) <= 64
    lo, hi = st._cache["bbox"]
    for t, s, a in zip(st.blk_tau, st.blk_sigma, st.blk_adm):
        assert bool(a) == trees.admissible(lo[t], hi[t], lo[s], hi[s])
    if n <= 2048:
        assert np.all(trees.coverage_bitmap(st) == 1)


@pytest.mark.parametrize("kind", ["hodlr", "blr"])
@pytest.mark.parametrize("n,seed", [(1, 1), (64, 2), (65, 3), (2048, 1001), (32768, 1002)])
def test_library_layout_equals_oracle(kind, n, seed):
    p = sphere_points(n, seed)
    st = trees.build_structure(p, kind=kind)
    e = hm.Layout(p, partition=kind).export()
    for k in ["perm", "begin", "end", "level", "parent", "son0", "son1", "blk_tau", "blk_sigma", "blk_adm"]:
        assert np.array_equal(e[k], getattr(st, k)), k


def case(kind, eps=1e-8):
    def build():
        p = sphere_points(2048, 1001)
        st = trees.build_structure(p, kind=kind)
        h = compress_h(p, KERNEL_LAPLACE, st, eps, method="svd")
        return p, st, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("partition", kind, eps), build)


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["hodlr", "blr"])
def test_products_within_truncation_bound(kind):
    """H products on the new partitions: three evaluation orders agree, and
    the product is within eps ||A||_F ||x|| of the dense kernel product (the
    exact-SVD bound of eq. 3 summed over blocks); UH and H^2 within 3 eps."""
    p, st, vals = case(kind)
    n = st.n
    x, y = gaussian_vector(n, 2001), gaussian_vector(n, 3001)
    h = vals["h"]
    a = mvm.h_mvm(st, h.dense, h.W, h.sigma, h.X, 1.0, x, y, order="block")
    b = mvm.h_mvm(st, h.dense, h.W, h.sigma, h.X, 1.0, x, y, order="rows")
    c = mvm.h_mvm(st, h.dense, h.W, h.sigma, h.X, 1.0, x, y, order="dense")
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a - y)
    assert np.linalg.norm(a - c) <= 1e-13 * np.linalg.norm(a - y)
    ref = dense.dense_product(KERNEL_LAPLACE, p, 1.0, x, y)
    fro = dense.kernel_fro_norm(KERNEL_LAPLACE, p)
    assert np.linalg.norm(a - ref) <= 1e-8 * fro * np.linalg.norm(x)
    u = vals["uh"]
    out = mvm.uh_mvm(st, u.dense, u.row_basis, u.col_basis, u.coupling, 1.0, x, y)
    assert np.linalg.norm(out - ref) <= 3e-8 * fro * np.linalg.norm(x)
    v = vals["h2"]
    out = mvm.h2_mvm(st, v.dense, v.row_rank, v.col_rank, v.row_leaf_basis, v.row_transfer, v.col_leaf_basis,
                     v.col_transfer, v.coupling, 1.0, x, y)
    assert np.linalg.norm(out - ref) <= 3e-8 * fro * np.linalg.norm(x)


def test_unknown_partition_is_rejected():
    from paper_2405_03456_amd import _lib
    import ctypes
    p = np.ascontiguousarray(sphere_points(100, 3))
    o = _lib.LayoutOpts(64, 2.0, 7)
    h = ctypes.c_void_p()
    st = _lib.lib().hm_build_layout(p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 100, ctypes.byref(o),
                                    ctypes.byref(h))
    assert st == _lib.HM_EINVAL
