"""Pins for the oracle's H / uniform-H / H^2 products and its dense product.

Each test fixes the oracle against something other than itself: closed forms
of special kernels, brute force on tiny inputs, the Eckart-Young error of a
truncated SVD, the eps bound of eq. 3 summed over blocks, and identities
between the three formats (Sec. 2.2-2.4, 3.1-3.3)."""
import numpy as np
import pytest

from conftest import cached
from oracle import dense, mvm, trees
from synth import (KERNEL_CONST, KERNEL_IDENTITY, KERNEL_LAPLACE, KERNEL_RANK1, compress_h,
                   gaussian_vector, rank1_factors, sphere_points, to_h2, to_uh)


def setup(n, kernel, eps, seed=1000, leaf=64):
    def make():
        p = sphere_points(n, seed)
        st = trees.build_structure(p, leaf)
        h = compress_h(p, kernel, st, eps, method="svd")
        return p, st, h
    return cached(("setup", n, kernel, eps, seed, leaf), make)


def hm(st, h, a, x, y, order="block"):
    return mvm.h_mvm(st, h.dense, h.W, h.sigma, h.X, a, x, y, order=order)


def rel(a, b, ref):
    return np.linalg.norm(a - b) / np.linalg.norm(ref)


# --------------------------------------------------------------- dense product

def test_dense_product_brute_force():
    p = sphere_points(37, 11)
    x = gaussian_vector(37, 12)
    y = gaussian_vector(37, 13)
    ref = y.copy()
    for i in range(37):
        s = 0.0
        for j in range(37):
            if i != j:
                d = p[i] - p[j]
                s += x[j] / (4 * np.pi * np.sqrt(d @ d))
        ref[i] += -0.5 * s
    for fn in (dense.dense_product, dense.dense_product_numpy):
        out = fn(KERNEL_LAPLACE, p, -0.5, x, y)
        assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()
    rows = np.array([3, 30, 5])
    out = dense.dense_product(KERNEL_LAPLACE, p, -0.5, x, y, rows=rows)
    assert np.array_equal(out[rows], ref[rows]) or np.abs(out[rows] - ref[rows]).max() < 1e-14
    others = np.setdiff1d(np.arange(37), rows)
    assert np.array_equal(out[others], y[others])


# ---------------------------------------------------------- closed forms (P-4)

@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_identity_kernel(fmt):
    n = 700
    p, st, h = setup(n, KERNEL_IDENTITY, 1e-10)
    assert all(h.rank(b) == 0 for b in range(st.nblocks) if st.blk_adm[b])
    x, y = gaussian_vector(n, 1), gaussian_vector(n, 2)
    out = run_format(fmt, st, h, -0.5, x, y)
    assert np.abs(out - (y - 0.5 * x)).max() < 1e-14


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_constant_kernel(fmt):
    n = 900
    p, st, h = setup(n, KERNEL_CONST, 1e-12)
    assert all(h.rank(b) == 1 for b in range(st.nblocks) if st.blk_adm[b])
    x, y = gaussian_vector(n, 3), gaussian_vector(n, 4)
    out = run_format(fmt, st, h, 1.0, x, y)
    ref = y + (x.sum() - x)
    assert np.abs(out - ref).max() < 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_rank1_kernel(fmt):
    n = 1000
    p, st, h = setup(n, KERNEL_RANK1, 1e-12)
    assert all(h.rank(b) == 1 for b in range(st.nblocks) if st.blk_adm[b])
    f, g = rank1_factors(p)
    x, y = gaussian_vector(n, 5), gaussian_vector(n, 6)
    out = run_format(fmt, st, h, 2.0, x, y)
    ref = y + 2.0 * (f * (g @ x) - f * g * x)
    assert np.abs(out - ref).max() < 1e-10 * np.abs(ref).max()
    if fmt == "uh":
        u = to_uh(h, st)
        assert max(b.shape[1] for b in u.row_basis) == 1


def run_format(fmt, st, h, a, x, y):
    if fmt == "h":
        return hm(st, h, a, x, y)
    if fmt == "uh":
        u = to_uh(h, st)
        return mvm.uh_mvm(st, u.dense, u.row_basis, u.col_basis, u.coupling, a, x, y)
    v = to_h2(h, st)
    return mvm.h2_mvm(st, v.dense, v.row_rank, v.col_rank, v.row_leaf_basis, v.row_transfer,
                      v.col_leaf_basis, v.col_transfer, v.coupling, a, x, y)


# -------------------------------------------------- brute force on tiny input

def test_h_brute_force_tiny():
    """n = 40, leaf 4: the H product equals a pure-Python double loop over
    the expanded blocks (no numpy products)."""
    p = sphere_points(40, 21)
    st = trees.build_structure(p, leaf_size=4)
    h = compress_h(p, KERNEL_LAPLACE, st, 1e-6, method="svd")
    assert st.blk_adm.any() and (~st.blk_adm).any()
    x, y = gaussian_vector(40, 22), gaussian_vector(40, 23)
    yc = [float(v) for v in y[st.perm]]
    xc = [float(v) for v in x[st.perm]]
    for b in range(st.nblocks):
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        for i in range(st.begin[t], st.end[t]):
            acc = 0.0
            for j in range(st.begin[s], st.end[s]):
                a, c = i - st.begin[t], j - st.begin[s]
                if st.blk_adm[b]:
                    e = sum(h.W[b][a, l] * h.sigma[b][l] * h.X[b][c, l] for l in range(h.rank(b)))
                else:
                    e = h.dense[b][a, c]
                acc += e * xc[j]
            yc[i] += 0.75 * acc
    ref = np.empty(40)
    ref[st.perm] = yc
    out = hm(st, h, 0.75, x, y)
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()


# ------------------------------------------------ evaluation orders (P-5)

@pytest.mark.parametrize("kernel", [KERNEL_LAPLACE])
def test_three_orders_agree(kernel):
    n = 2048
    p, st, h = setup(n, kernel, 1e-8, seed=1001)
    x, y = gaussian_vector(n, 2001), gaussian_vector(n, 3001)
    a = hm(st, h, 1.0, x, y, "block")
    b = hm(st, h, 1.0, x, y, "rows")
    c = hm(st, h, 1.0, x, y, "dense")
    assert rel(a, b, a - y) < 1e-13 and rel(a, c, a - y) < 1e-13
    u = to_uh(h, st)
    a = mvm.uh_mvm(st, u.dense, u.row_basis, u.col_basis, u.coupling, 1.0, x, y, "phases")
    b = mvm.uh_mvm(st, u.dense, u.row_basis, u.col_basis, u.coupling, 1.0, x, y, "rows")
    c = mvm.uh_mvm(st, u.dense, u.row_basis, u.col_basis, u.coupling, 1.0, x, y, "dense")
    assert rel(a, b, a - y) < 1e-13 and rel(a, c, a - y) < 1e-13


# ------------------------------------------------ truncation bounds (P-3)

def test_eckart_young_per_block():
    n = 2048
    p, st, h = setup(n, KERNEL_LAPLACE, 1e-8, seed=1001)
    from synth.hmatrix import dense_block
    pc = p[st.perm]
    checked = 0
    for b in np.nonzero(st.blk_adm)[0][::7]:
        M = dense_block(pc, KERNEL_LAPLACE, st, int(b))
        s = np.linalg.svd(M, compute_uv=False)
        k = h.rank(b)
        err = np.linalg.norm(M - (h.W[b] * h.sigma[b]) @ h.X[b].T)
        tail = np.sqrt((s[k:] ** 2).sum())
        assert abs(err - tail) <= 1e-12 * np.linalg.norm(M) + 1e-3 * tail
        assert tail <= 1e-8 * np.linalg.norm(M) * (1 + 1e-12)
        if k > 0:   # k is the smallest admissible rank
            assert np.sqrt((s[k - 1:] ** 2).sum()) > 1e-8 * np.linalg.norm(M)
        checked += 1
    assert checked > 50


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_global_eps_bound(eps):
    """||A - A_H||_F <= eps ||A||_F, hence ||y_H - y_dense|| <= eps ||A||_F ||x||."""
    n = 2048
    p, st, h = setup(n, KERNEL_LAPLACE, eps, seed=1001)
    x, y = gaussian_vector(n, 2001), gaussian_vector(n, 3001)
    yh = hm(st, h, 1.0, x, y)
    yd = dense.dense_product(KERNEL_LAPLACE, p, 1.0, x, y)
    fro = dense.kernel_fro_norm(KERNEL_LAPLACE, p)
    assert np.linalg.norm(yh - yd) <= eps * fro * np.linalg.norm(x)
    # statistically E||Ax||^2 = ||A||_F^2: the relative error is of order eps
    assert rel(yh, yd, yd - y) < 5 * eps


# ------------------------------------------------ format identities (P-6)

def test_uh_and_h2_structure():
    n = 2048
    eps = 1e-6
    p, st, h = setup(n, KERNEL_LAPLACE, eps, seed=1001)
    u = to_uh(h, st)
    for v in range(st.nnodes):
        B = u.row_basis[v]
        if B.shape[1]:
            assert np.abs(B.T @ B - np.eye(B.shape[1])).max() < 1e-12
    for b in np.nonzero(st.blk_adm)[0]:
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        Mh = (h.W[b] * h.sigma[b]) @ h.X[b].T
        Mu = u.row_basis[t] @ u.coupling[b] @ u.col_basis[s].T
        assert np.linalg.norm(Mh - Mu) <= 3 * eps * np.linalg.norm(Mh) + 1e-300
    v2 = to_h2(h, st)
    rb = mvm.h2_explicit_bases(st, v2.row_leaf_basis, v2.row_transfer)
    for v in range(st.nnodes):
        if rb[v].shape[1]:
            assert np.abs(rb[v].T @ rb[v] - np.eye(rb[v].shape[1])).max() < 1e-12
        if not st.is_leaf(v):      # nestedness: W_t = [W_t0 E_t0; W_t1 E_t1]
            a, c = st.sons(v)
            assert np.allclose(rb[v], np.vstack([rb[a] @ v2.row_transfer[a],
                                                 rb[c] @ v2.row_transfer[c]]), atol=1e-13)
    x, y = gaussian_vector(n, 2), gaussian_vector(n, 3)
    args = (st, v2.dense, v2.row_rank, v2.col_rank, v2.row_leaf_basis, v2.row_transfer,
            v2.col_leaf_basis, v2.col_transfer, v2.coupling, 1.0, x, y)
    a = mvm.h2_mvm(*args)
    b = mvm.h2_mvm(*args, order="via_uh")
    assert rel(a, b, a - y) < 1e-13
    yd = dense.dense_product(KERNEL_LAPLACE, p, 1.0, x, y)
    assert rel(a, yd, yd - y) < 20 * eps


def test_linearity_and_many_rhs():
    n = 2048
    p, st, h = setup(n, KERNEL_LAPLACE, 1e-8, seed=1001)
    x1, x2, y = gaussian_vector(n, 1), gaussian_vector(n, 2), np.zeros(n)
    lhs = hm(st, h, 1.0, 2.0 * x1 - 3.0 * x2, y)
    rhs = 2.0 * hm(st, h, 1.0, x1, y) - 3.0 * hm(st, h, 1.0, x2, y)
    assert rel(lhs, rhs, lhs) < 1e-13
    X = np.stack([x1, x2], axis=1)
    Y = np.stack([y, y + 1], axis=1)
    out = mvm.columns(mvm.h_mvm, X, Y, st, h.dense, h.W, h.sigma, h.X, 1.0)
    assert np.array_equal(out[:, 1], hm(st, h, 1.0, x2, y + 1))


def test_planted_mistake_is_caught():
    """A dropped low-rank term (planted in a copy of the factors) must break
    agreement with the dense product by far more than eps."""
    n = 2048
    p, st, h = setup(n, KERNEL_LAPLACE, 1e-8, seed=1001)
    x, y = gaussian_vector(n, 1), np.zeros(n)
    W = list(h.W)
    b = int(np.nonzero(st.blk_adm)[0][0])
    W[b] = W[b].copy(); W[b][:, 0] = 0.0
    bad = mvm.h_mvm(st, h.dense, W, h.sigma, h.X, 1.0, x, y)
    yd = dense.dense_product(KERNEL_LAPLACE, p, 1.0, x, y)
    assert rel(bad, yd, yd) > 1e-6


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_product_many_closed_forms(fmt):
    """Many right-hand sides (one product per column): identity kernel gives
    Y + alpha X, constant kernel Y + alpha (column sums - X)."""
    from oracle import stored
    from synth import gaussian_matrix
    for kernel, n in ((KERNEL_IDENTITY, 700), (KERNEL_CONST, 900)):
        p, st, h = setup(n, kernel, 1e-10 if kernel == KERNEL_IDENTITY else 1e-12)
        vals = {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}[fmt]
        X, Y = gaussian_matrix(n, 5, 11), gaussian_matrix(n, 5, 12)
        out = stored.product_many(st, fmt, vals, -0.5, X, Y)
        ref = Y - 0.5 * (X if kernel == KERNEL_IDENTITY else X.sum(axis=0)[None, :] - X)
        assert np.abs(out - ref).max() < 1e-11 * np.abs(ref).max()
