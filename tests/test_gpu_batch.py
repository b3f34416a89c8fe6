"""GPU parity of the many-right-hand-side path (hm_mvm_batch) against the
oracle, column by column, on the same stored matrix.

Tolerances (relative L2 of each column's increment):
  * float64 data and float64 accumulation (float64 MFMA): 1e-10;
  * float32 accumulation (float32 MFMA on the stored values): 1e-6;
  * float32 vectors: the oracle gets X rounded to float32; 1e-6.
Widths cover one 16-wide block, a ragged block, several 64-wide blocks and
a ragged tail; the leading dimensions differ from n."""
import numpy as np
import pytest

from conftest import cached
from oracle import stored, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_matrix, sphere_points, to_h2, to_uh

pytestmark = pytest.mark.gpu

POLICIES = {
    "f64": (dict(dense="f64", factor="f64", eps=1e-8), 1e-10),
    "f32": (dict(dense="f32", factor="f32", eps=1e-6), 1e-6),
    "bf16": (dict(dense="f32", diag="f64", factor="bf16", coupling="f32", eps=1e-6), 1e-6),
    "fp8": (dict(dense="f32", diag="f64", factor="fp8", coupling="fp8", eps=1e-6), 1e-6),
    "valr6": (dict(dense="valr", diag="valr", factor="valr", eps=1e-6), 1e-6),
    "valr8": (dict(dense="valr", diag="valr", factor="valr", eps=1e-8), 1e-10),
}


def case(n=2048, seed=1001):
    def build():
        import paper_2405_03456_amd as hm
        p = sphere_points(n, seed)
        st = trees.build_structure(p)
        lay = hm.Layout(p)
        h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
        return st, lay, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("batch", n, seed), build)


def colerr(out, ref, y0):
    d = np.linalg.norm(out - ref, axis=0)
    s = np.maximum(np.linalg.norm(ref - y0, axis=0), 1e-300)
    return (d / s).max()


def padded(torch, A, ld, dtype):
    """A column-major device copy of A with leading dimension ld >= n."""
    n, r = A.shape
    buf = torch.zeros((r, ld), dtype=dtype, device="cuda")
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(A.T)).to(dtype)
    return buf.T[:n, :]


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", list(POLICIES))
@pytest.mark.parametrize("r", [5, 16, 33, 130])
def test_batch_parity(fmt, pol, r):
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, tol = POLICIES[pol]
    n = st.n
    print(f"case batch fmt={fmt} policy={pol} r={r}", flush=True)
    X, Y = gaussian_matrix(n, r, 2000 + r), gaussian_matrix(n, r, 3000 + r)
    sv = stored.stored_values(st, fmt, vals[fmt], dense=pp["dense"], diag=pp.get("diag"),
                              factor=pp["factor"], coupling=pp.get("coupling"), eps=pp["eps"])
    ref = stored.product_many(st, fmt, sv, -0.5, X, Y)
    M = hm.Matrix(lay, fmt, vals[fmt], **pp)
    Xd, Yd = padded(torch, X, n + 7, torch.float64), padded(torch, Y, n + 3, torch.float64)
    M.mvm_many(Xd, Yd, alpha=-0.5)
    torch.cuda.synchronize()
    err = colerr(Yd.cpu().numpy(), ref, Y)
    print(f"  worst column rel err {err:.3e} (tol {tol:g})", flush=True)
    M.free()
    assert err <= tol


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_batch_f32_vectors_and_cluster_order(fmt):
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    n, r = st.n, 24
    pp = POLICIES["f32"][0]
    X = gaussian_matrix(n, r, 7).astype(np.float32).astype(np.float64)
    Y = gaussian_matrix(n, r, 8).astype(np.float32).astype(np.float64)
    sv = stored.stored_values(st, fmt, vals[fmt], dense="f32", factor="f32", eps=1e-6)
    ref = stored.product_many(st, fmt, sv, 1.0, X, Y)
    M = hm.Matrix(lay, fmt, vals[fmt], **pp)
    Xd, Yd = padded(torch, X, n, torch.float32), padded(torch, Y, n, torch.float32)
    M.mvm_many(Xd, Yd)
    # cluster order: the same product on permuted vectors
    Xc, Yc = padded(torch, X[st.perm], n, torch.float64), padded(torch, Y[st.perm], n, torch.float64)
    M.mvm_many(Xc, Yc, cluster_order=True)
    torch.cuda.synchronize()
    assert colerr(Yd.double().cpu().numpy(), ref, Y) <= 1e-6
    assert colerr(Yc.cpu().numpy(), ref[st.perm], Y[st.perm]) <= 1e-6
    M.free()


def test_batch_several_matrices_one_call():
    """Three matrices of different formats and widths in one hm_mvm_batch,
    including a width-1 float64 entry (the single-vector kernels) and an
    empty one; each result equals its own single-matrix call bitwise."""
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    n = st.n
    pp = POLICIES["valr6"][0]
    Ms = [hm.Matrix(lay, f, vals[f], **pp) for f in ("h", "uh", "h2", "h")]
    widths = [1, 40, 17, 0]
    Xs = [padded(torch, gaussian_matrix(n, max(r, 1), 40 + i), n, torch.float64)[:, :r] for i, r in enumerate(widths)]
    Ys = [padded(torch, gaussian_matrix(n, max(r, 1), 50 + i), n, torch.float64)[:, :r] for i, r in enumerate(widths)]
    Y0 = [y.clone() for y in Ys]
    hm.mvm_batch(Ms, Xs, Ys, alpha=0.75)
    for M, x, y in zip(Ms[:3], Xs[:3], Y0[:3]):
        if x.shape[1] == 1:
            yy = y[:, 0].contiguous()
            M.mvm(x[:, 0].contiguous(), yy, alpha=0.75)
            y[:, 0] = yy
        else:
            M.mvm_many(x, y, alpha=0.75)
    torch.cuda.synchronize()
    for i in range(3):
        assert torch.equal(Ys[i], Y0[i]), i
    for M in Ms:
        M.free()


def test_batch_errors():
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    n = st.n
    M = hm.Matrix(lay, "h", vals["h"], dense="f32", factor="f32", eps=1e-6)
    X = torch.zeros((n, 4), dtype=torch.float64, device="cuda")   # row-major: rejected by the binding
    with pytest.raises(ValueError):
        M.mvm_many(X, X.clone())
    Xc = padded(torch, np.zeros((n, 4)), n, torch.float64)
    with pytest.raises(hm.HMError):                                 # the same matrix twice
        hm.mvm_batch([M, M], [Xc, Xc.clone()], [Xc.clone(), Xc.clone()])
    with pytest.raises(hm.HMError):                                 # X == Y
        hm.mvm_batch([M], [Xc], [Xc])
    M.free()


def test_batch_graph_replays_and_timing():
    """A captured hm_mvm_batch replays bitwise like the eager call, with
    unrelated torch work and synchronisations between replays; HM_TIMING
    reports per-phase times at the block width."""
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    n = st.n
    Ms = [hm.Matrix(lay, f, vals[f], dense="f32", diag="f64", factor="bf16", coupling="f32", eps=1e-6)
          for f in ("uh", "h2")]
    Xs = [padded(torch, gaussian_matrix(n, r, 60 + r), n, torch.float64) for r in (20, 70)]
    Ye = [torch.zeros_like(x) for x in Xs]
    hm.mvm_batch(Ms, Xs, Ye, alpha=1.5)
    Yg = [torch.zeros_like(x) for x in Xs]
    g = hm.BatchGraph(Ms, Xs, Yg, alpha=1.5)
    for rep in range(3):
        for y in Yg:
            y.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()      # unrelated work between replays
        g.launch()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a, b in zip(Yg, Ye):
            assert torch.equal(a, b), rep
    g.free()
    Ms[0].mvm_many(Xs[0], Ye[0], timing=True)
    ph = Ms[0].timing()
    assert all(p["nrhs"] == 32 for p in ph if p["launches"] > 0)
    assert sum(p["launches"] for p in ph) > 0 and all(p["ms_total"] >= 0 for p in ph)
    for M in Ms:
        M.free()


@pytest.mark.parametrize("fmt", ["h", "h2"])
def test_tuner_keeps_parity(fmt):
    """hm_tune_batch times every plan candidate and keeps the fastest; the
    product stays within the accumulation tolerance of the oracle."""
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    n, r = st.n, 40
    pp, tol = POLICIES["bf16"]
    M = hm.Matrix(lay, fmt, vals[fmt], **pp)
    res = M.tune(r, reps=2)
    assert res["ncandidates"] == 15 and res["nrb"] in (1, 2) and res["ms"] > 0
    assert 64 * 1024 <= res["target_bytes"] <= 1024 * 1024
    X, Y = gaussian_matrix(n, r, 91), gaussian_matrix(n, r, 92)
    sv = stored.stored_values(st, fmt, vals[fmt], dense=pp["dense"], diag=pp.get("diag"),
                              factor=pp["factor"], coupling=pp.get("coupling"), eps=pp["eps"])
    ref = stored.product_many(st, fmt, sv, 1.0, X, Y)
    Xd, Yd = padded(torch, X, n, torch.float64), padded(torch, Y, n, torch.float64)
    M.mvm_many(Xd, Yd)
    torch.cuda.synchronize()
    assert colerr(Yd.cpu().numpy(), ref, Y) <= tol
    M.free()


def test_batch_many_matrices_merged_launches():
    """26 matrices (more than one launch's job table) of mixed formats,
    storage and widths in one call: each result equals its own call bitwise."""
    import torch
    import paper_2405_03456_amd as hm
    n = 300
    p = sphere_points(n, 77)
    st = trees.build_structure(p)
    lay = hm.Layout(p)
    h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
    vals = {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    pols = [POLICIES[k][0] for k in ("f64", "f32", "bf16", "valr6")]
    Ms, Xs, Ys = [], [], []
    for i in range(26):
        fmt = ("h", "uh", "h2")[i % 3]
        Ms.append(hm.Matrix(lay, fmt, vals[fmt], **pols[i % 4]))
        r = 2 + (7 * i) % 39
        Xs.append(padded(torch, gaussian_matrix(n, r, 500 + i), n, torch.float64))
        Ys.append(padded(torch, gaussian_matrix(n, r, 600 + i), n, torch.float64))
    Y0 = [y.clone() for y in Ys]
    hm.mvm_batch(Ms, Xs, Ys, alpha=-1.25)
    for M, x, y in zip(Ms, Xs, Y0):
        M.mvm_many(x, y, alpha=-1.25)
    torch.cuda.synchronize()
    for i in range(26):
        assert torch.equal(Ys[i], Y0[i]), i
    for M in Ms:
        M.free()


def test_batch_maximum_width_and_beyond():
    """HM_MAX_NRHS columns in one call match the oracle column by column;
    one column more is rejected before anything runs."""
    import torch
    import paper_2405_03456_amd as hm
    n = 300
    p = sphere_points(n, 79)
    st = trees.build_structure(p)
    lay = hm.Layout(p)
    h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
    vals = {"h": h, "uh": to_uh(h, st)}
    pp, tol = POLICIES["f32"]
    for fmt in ("h", "uh"):
        M = hm.Matrix(lay, fmt, vals[fmt], **pp)
        r = 1024
        X, Y = gaussian_matrix(n, r, 700), gaussian_matrix(n, r, 701)
        sv = stored.stored_values(st, fmt, vals[fmt], dense=pp["dense"], factor=pp["factor"], eps=pp["eps"])
        ref = stored.product_many(st, fmt, sv, 0.5, X, Y)
        Xd, Yd = padded(torch, X, n, torch.float64), padded(torch, Y, n, torch.float64)
        M.mvm_many(Xd, Yd, alpha=0.5)
        torch.cuda.synchronize()
        assert colerr(Yd.cpu().numpy(), ref, Y) <= tol, fmt
        Xb = padded(torch, np.zeros((n, r + 1)), n, torch.float64)
        Yb = padded(torch, np.zeros((n, r + 1)), n, torch.float64)
        with pytest.raises(hm.HMError):
            M.mvm_many(Xb, Yb)
        M.free()


def test_stale_batch_graph_is_refused():
    """A batch graph holds device addresses of its matrix's many-RHS
    workspace: after a wider product regrows that workspace the graph is
    refused (HM_EINVAL) before anything is launched, and a graph captured
    afterwards replays correctly."""
    import torch
    import paper_2405_03456_amd as hm
    from paper_2405_03456_amd import _lib
    st, lay, vals = case()
    print("case stale batch graph h n=2048 r=16 -> 64", flush=True)
    pol, tol = POLICIES["f32"]
    M = hm.Matrix(lay, "h", vals["h"], **pol)
    X = gaussian_matrix(st.n, 64, 77)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda().T
    Y16 = torch.zeros((16, st.n), dtype=torch.float64, device="cuda").T
    g = hm.BatchGraph([M], [Xd[:, :16]], [Y16])
    g.launch()
    Y64 = torch.zeros((64, st.n), dtype=torch.float64, device="cuda").T
    hm.mvm_batch([M], [Xd], [Y64])              # grows the workspace to 64 columns
    torch.cuda.synchronize()
    before = Y16.clone()
    with pytest.raises(hm.HMError) as ex:
        g.launch()
    assert ex.value.status == _lib.HM_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(before, Y16)              # nothing ran
    g.free()
    g2 = hm.BatchGraph([M], [Xd[:, :16]], [Y16])
    g2.launch()
    torch.cuda.synchronize()
    sv = stored.stored_values(st, "h", vals["h"], dense=pol["dense"], factor=pol["factor"], eps=pol["eps"])
    ref = stored.product_many(st, "h", sv, 1.0, X[:, :16], np.zeros((st.n, 16)))
    assert colerr(Y16.cpu().numpy() / 2.0, ref, 0.0) <= tol
    g2.free()
    M.free()
