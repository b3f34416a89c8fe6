"""GPU parity: the HIP product against the oracle on the same stored matrix.

Tolerances (relative L2 of the increment y_out - y_in):
  * float64 storage and float64 accumulation: 1e-10,
  * every other policy: 1e-6 (float32 accumulation; the oracle sees the
    dequantised stored values exactly, so only accumulation order and the
    float32 products differ, Sec. 4.1/4.2 storage error is not part of it).
The layout and the oracle's trees are compared bit for bit before use."""
import numpy as np
import pytest

from conftest import cached
from oracle import stored, trees
from synth import (KERNEL_IDENTITY, KERNEL_LAPLACE, compress_h, gaussian_vector, sphere_points,
                   to_h2, to_uh)

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-6


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def make(n, eps, kernel=KERNEL_LAPLACE, seed=1001, leaf=64):
    def build():
        import paper_2405_03456_amd as hm
        p = sphere_points(n, seed)
        st = trees.build_structure(p, leaf)
        lay = hm.Layout(p, leaf_size=leaf)
        e = lay.export()
        for k in ["perm", "begin", "end", "blk_tau", "blk_sigma", "blk_adm"]:
            assert np.array_equal(e[k], getattr(st, k))
        h = compress_h(p, kernel, st, eps, method="svd" if n <= 8192 else "auto")
        vals = {"h": h}
        if kernel != KERNEL_IDENTITY or True:
            vals["uh"] = to_uh(h, st)
            vals["h2"] = to_h2(h, st)
        return p, st, lay, vals
    return cached(("gpu", n, eps, kernel, seed, leaf), build)


def run_gpu(lay, fmt, values, x, y, alpha, cluster=False, **policy):
    import paper_2405_03456_amd as hm
    torch = torch_cuda()
    M = hm.Matrix(lay, fmt, values, **policy)
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, yd, alpha=alpha, cluster_order=cluster)
    torch.cuda.synchronize()
    out = yd.cpu().numpy()
    M.free()
    return out


def rel(a, b, y0):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b - y0), 1e-300)


POLICIES = {
    "f64": dict(dense="f64", factor="f64", eps=1e-8),
    "f32": dict(dense="f32", factor="f32", eps=1e-6),
    "bf16": dict(dense="f32", diag="f64", factor="bf16", coupling="f32", eps=1e-6),
    "f16": dict(dense="f32", diag="f64", factor="f16", coupling="f16", eps=1e-6),
    "fp8": dict(dense="f32", diag="f64", factor="fp8", coupling="fp8", eps=1e-6),
    "f32acc64": dict(dense="f32", factor="f32", eps=1e-8),
    # VALR (Sec. 4.2): per-column formats of factors/bases, direct dense and
    # coupling formats at eps, FP64 diagonal near field
    "valr4": dict(dense="valr", diag="valr", factor="valr", eps=1e-4),
    "valr6": dict(dense="valr", diag="valr", factor="valr", eps=1e-6),
    "valr8": dict(dense="valr", diag="valr", factor="valr", eps=1e-8),
}
ACC64 = ("f64", "f32acc64", "valr8")


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", list(POLICIES))
def test_parity_n2048(fmt, pol):
    n = 2048
    p, st, lay, vals = make(n, 1e-8)
    pp = dict(POLICIES[pol])
    print(f"case fmt={fmt} policy={pol} n={n}", flush=True)
    x, y = gaussian_vector(n, 2001), gaussian_vector(n, 3001)
    sv = stored.stored_values(st, fmt, vals[fmt], dense=pp["dense"], diag=pp.get("diag"),
                              factor=pp["factor"], coupling=pp.get("coupling"), eps=pp["eps"])
    ref = stored.product(st, fmt, sv, -0.5, x, y)
    out = run_gpu(lay, fmt, vals[fmt], x, y, -0.5, **pp)
    tol = TOL64 if pol in ACC64 else TOL32
    err = rel(out, ref, y)
    print(f"  rel err {err:.3e} (tol {tol:g})", flush=True)
    assert err <= tol


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_cluster_order_and_determinism(fmt):
    n = 2048
    p, st, lay, vals = make(n, 1e-8)
    x, y = gaussian_vector(n, 5), gaussian_vector(n, 6)
    a = run_gpu(lay, fmt, vals[fmt], x, y, 1.0)
    b = run_gpu(lay, fmt, vals[fmt], x, y, 1.0)
    assert np.array_equal(a, b)                      # bitwise reproducible
    c = run_gpu(lay, fmt, vals[fmt], x[st.perm], y[st.perm], 1.0, cluster=True)
    assert np.array_equal(c, a[st.perm])


@pytest.mark.parametrize("n", [1, 64, 65, 300])
def test_small_and_ragged(n):
    p, st, lay, vals = make(n, 1e-10, seed=77)
    x, y = gaussian_vector(n, 8), gaussian_vector(n, 9)
    for fmt in ("h", "uh", "h2"):
        ref = stored.product(st, fmt, vals[fmt], 2.0, x, y)
        out = run_gpu(lay, fmt, vals[fmt], x, y, 2.0)
        assert rel(out, ref, y) <= TOL64, (n, fmt)


def test_identity_kernel_rank_zero_blocks():
    n = 1500
    p, st, lay, vals = make(n, 1e-10, kernel=KERNEL_IDENTITY, seed=78)
    x, y = gaussian_vector(n, 10), gaussian_vector(n, 11)
    for fmt in ("h", "uh", "h2"):
        out = run_gpu(lay, fmt, vals[fmt], x, y, -0.5)
        assert np.array_equal(out, y - 0.5 * x), fmt


@pytest.mark.parametrize("fmt", ["uh", "h2"])
def test_tune_mvm_keeps_results_bitwise(fmt):
    """hm_tune_mvm times every fork point of the dense stage (staged
    schedule) and a spread of interleave points of the dense tasks
    (persistent schedule) and keeps the fastest; both move work in time
    only, so eager products and graph replays after tuning equal the untuned
    product bit for bit."""
    import paper_2405_03456_amd as hm
    torch = torch_cuda()
    n = 2048
    p, st, lay, vals = make(n, 1e-8)
    x, y = gaussian_vector(n, 12), gaussian_vector(n, 13)
    M = hm.Matrix(lay, fmt, vals[fmt], dense="valr", diag="valr", factor="valr", eps=1e-6, schedule="persistent")
    xd = torch.from_numpy(x).cuda()
    y0 = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, y0, alpha=0.5)
    r = M.tune_mvm(reps=3)
    # staged: one candidate per fork point 0 ... number of chain stages with
    # tasks, for each of four caps on the dense stage's workgroups (none, 1,
    # 2 and 3 per compute unit); persistent: at most 17 interleave points
    nchain = sum(1 for ph in M.timing() if ph["ntasks"] > 0 and ph["name"] not in ("dense", "persistent"))
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    # (+ at most 24 split candidates: 8 second fork points x 3 fractions)
    nstaged = 4 * (nchain + 1)
    assert nstaged + 1 <= r["ncandidates"] <= nstaged + 24 + 17 and 0 <= r["fork_after"] <= nchain
    assert r["dense_grid"] in (0, ncu, 2 * ncu, 3 * ncu)
    assert r["dense_split"] == 0 or (r["schedule"] == "staged" and r["fork2"] > r["fork_after"])
    assert r["ms"] > 0 and r["ms"] <= r["ms_first"] and r["ms"] == min(r["ms_staged"], r["ms_persistent"])
    assert r["schedule"] == ("staged" if r["ms"] == r["ms_staged"] else "persistent")
    M.check()
    y1 = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, y1, alpha=0.5)
    y2 = torch.from_numpy(y.copy()).cuda()
    g = M.graph(xd, y2, alpha=0.5)
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(y0, y1) and torch.equal(y0, y2)
    g.free()
    M.free()


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", ["f64", "valr6"])
def test_parity_small_tasks(fmt, pol):
    """2000-byte tasks split coefficient owners into many tasks: stages whose
    owners exceed the deferral limit keep their reduction launch, the others
    are summed by their consumers; both against the oracle."""
    n = 2048
    p, st, lay, vals = make(n, 1e-8)
    pp = dict(POLICIES[pol])
    x, y = gaussian_vector(n, 2101), gaussian_vector(n, 3101)
    sv = stored.stored_values(st, fmt, vals[fmt], dense=pp["dense"], diag=pp.get("diag"),
                              factor=pp["factor"], coupling=pp.get("coupling"), eps=pp["eps"])
    ref = stored.product(st, fmt, sv, 0.75, x, y)
    out = run_gpu(lay, fmt, vals[fmt], x, y, 0.75, task_bytes=2000, **pp)
    tol = TOL64 if pol in ACC64 else TOL32
    assert rel(out, ref, y) <= tol


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_valr_tile_promotion_within_budget(fmt, eps):
    """The library's optional tile promotion (valr_promote) stores some
    columns more precisely than Sec. 4.2 asks.  Its product is checked
    against the oracle's paper rule (every column in its own cheapest
    format): the two stored matrices differ by at most the VALR budgets, so
    the products agree within a small multiple of eps (eq. 6 / eq. 7), as
    does the promoted product and the float64 product."""
    n = 2048
    p, st, lay, vals = make(n, 1e-8)
    print(f"case valr promotion {fmt} eps={eps:g}", flush=True)
    x, y = gaussian_vector(n, 2201), gaussian_vector(n, 3201)
    pol = dict(dense="valr", diag="valr", factor="valr", eps=eps)
    sv = stored.stored_values(st, fmt, vals[fmt], **pol)
    ref = stored.product(st, fmt, sv, 1.0, x, y)
    exact = stored.product(st, fmt, vals[fmt], 1.0, x, y)
    out = run_gpu(lay, fmt, vals[fmt], x, y, 1.0, valr_promote=True, **pol)
    plain = run_gpu(lay, fmt, vals[fmt], x, y, 1.0, **pol)
    assert rel(plain, ref, y) <= TOL32                       # paper rule: parity
    assert rel(out, ref, y) <= 3.0 * eps                     # promotion: within the budget
    assert rel(out, exact, y) <= 3.0 * eps                   # ... of the float64 product too


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_split_dense_stage_is_bitwise_neutral(fmt):
    """The dense stage as two launches (hm_set_dense_split) at several split
    points and second fork points: eager products and graph replays equal
    the one-launch product bit for bit, and per-phase timing counts the two
    launches as one per product."""
    import paper_2405_03456_amd as hm
    torch = torch_cuda()
    n = 2048
    p, st, lay, vals = make(n, 1e-8)
    x, y = gaussian_vector(n, 22), gaussian_vector(n, 23)
    print(f"case split dense stage {fmt}", flush=True)
    M = hm.Matrix(lay, fmt, vals[fmt], dense="f64", factor="f64", eps=1e-8)
    xd = torch.from_numpy(x).cuda()
    y0 = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, y0, alpha=-1.5)
    nd = sum(ph["ntasks"] for ph in M.timing() if ph["name"] == "dense")
    nchain = sum(1 for ph in M.timing() if ph["ntasks"] > 0 and ph["name"] != "dense")
    assert nd >= 4
    for f2 in (0, 1, nchain, nchain + 5):
        for first in (1, nd // 2, nd - 1):
            M.set_dense_split(f2, first)
            y1 = torch.from_numpy(y.copy()).cuda()
            M.mvm(xd, y1, alpha=-1.5, timing=True)
            y2 = torch.from_numpy(y.copy()).cuda()
            g = M.graph(xd, y2, alpha=-1.5)
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(y0, y1) and torch.equal(y0, y2), (f2, first)
            g.free()
            dense = [ph for ph in M.timing() if ph["name"] == "dense"][0]
            assert dense["launches"] == 1
    with pytest.raises(hm.HMError):
        M.set_dense_split(1, nd)
    M.set_dense_split(0, 0)
    M.free()
