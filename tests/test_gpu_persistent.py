"""GPU tests of the persistent schedule (one launch running the plan's tasks
from a ticket queue, each task waiting only for the owners it reads).

It runs exactly the arithmetic of the one-launch-per-stage schedule, so the
two are compared bitwise, for every format, storage policy and task size
(small tasks split owners: deferred partial sums and reduction items), and
both against the oracle.  Also: repeated products and graph replays are
bitwise identical (the order in which waves take tickets varies, the
arithmetic of every output does not), every interleave point of the dense
tasks gives the same result, and a wait bound too small to be met ends the
launch and is reported by hm_matrix_check instead of hanging."""
import numpy as np
import pytest

from conftest import cached
from oracle import stored, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_vector, sphere_points, to_h2, to_uh

pytestmark = pytest.mark.gpu

POLICIES = {
    "f64": (dict(dense="f64", factor="f64", eps=1e-8), 1e-10),
    "f32": (dict(dense="f32", factor="f32", eps=1e-6), 1e-6),
    "bf16": (dict(dense="f32", diag="f64", factor="bf16", coupling="bf16", eps=1e-6), 1e-6),
    "fp8": (dict(dense="f32", diag="f64", factor="fp8", coupling="fp8", eps=1e-6), 1e-6),
    "valr6": (dict(dense="valr", diag="valr", factor="valr", eps=1e-6), 1e-6),
}


def case(n=2048, seed=1001):
    def build():
        import paper_2405_03456_amd as hm
        p = sphere_points(n, seed)
        st = trees.build_structure(p)
        lay = hm.Layout(p)
        h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
        return st, lay, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("persist", n, seed), build)


def product(M, x, y, alpha=0.75):
    import torch
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, yd, alpha=alpha)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", list(POLICIES))
@pytest.mark.parametrize("tb", [0, 2000])
def test_persistent_equals_staged(fmt, pol, tb):
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, tol = POLICIES[pol]
    print(f"case persistent vs staged {fmt} {pol} task_bytes={tb}", flush=True)
    x, y = gaussian_vector(st.n, 2301), gaussian_vector(st.n, 3301)
    Mp = hm.Matrix(lay, fmt, vals[fmt], task_bytes=tb, schedule="persistent", **pp)
    Ms = hm.Matrix(lay, fmt, vals[fmt], task_bytes=tb, schedule="staged", **pp)
    assert Mp.stats()["nlaunch"] == 2 and Ms.stats()["nlaunch"] > 2
    assert hm.Matrix(lay, fmt, vals[fmt], task_bytes=tb, **pp).stats()["nlaunch"] > 2   # staged by default
    a = product(Mp, x, y)
    b = product(Ms, x, y)
    Mp.check()
    assert np.array_equal(a, b)
    sv = stored.stored_values(st, fmt, vals[fmt], dense=pp["dense"], diag=pp.get("diag"), factor=pp["factor"],
                              coupling=pp.get("coupling"), eps=pp["eps"])
    ref = stored.product(st, fmt, sv, 0.75, x, y)
    assert np.linalg.norm(a - ref) / np.linalg.norm(ref - y) <= tol
    Mp.free()
    Ms.free()


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_persistent_repeatable_graphs_and_interleave(fmt):
    """Ten products and ten graph replays bitwise equal to the first
    product; every dense interleave point (set at upload) gives the same
    bits; the tuner picks a schedule without changing them."""
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, _ = POLICIES["valr6"]
    print(f"case persistent repeat/graph/interleave {fmt}", flush=True)
    x, y = gaussian_vector(st.n, 2401), gaussian_vector(st.n, 3401)
    M = hm.Matrix(lay, fmt, vals[fmt], task_bytes=4000, schedule="persistent", **pp)
    first = product(M, x, y)
    for _ in range(10):
        assert np.array_equal(product(M, x, y), first)
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y.copy()).cuda()
    g = M.graph(xd, yd, alpha=0.75)
    for _ in range(10):
        yd.copy_(torch.from_numpy(y))
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(yd.cpu().numpy(), first)
    g.free()
    M.check()
    for da in (1, 2, 5, 100):
        Md = hm.Matrix(lay, fmt, vals[fmt], task_bytes=4000, dense_after=da, schedule="persistent", **pp)
        assert np.array_equal(product(Md, x, y), first), da
        Md.check()
        Md.free()
    r = M.tune_mvm(reps=3)
    assert r["ms"] > 0 and r["schedule"] in ("staged", "persistent")
    assert np.array_equal(product(M, x, y), first)
    M.check()
    M.free()


def test_wait_bound_ends_the_launch():
    """A 1-microsecond bound on a dependency wait: launches that have to
    wait abort instead of waiting (every kernel still ends), the abort is
    reported by hm_matrix_check, and the matrix works again afterwards once
    waits are allowed (a fresh upload with the default bound)."""
    import paper_2405_03456_amd as hm
    from paper_2405_03456_amd import _lib
    st, lay, vals = case()
    pp, tol = POLICIES["f64"]
    print("case persistent wait bound 1 us (h2, 2000-byte tasks)", flush=True)
    x, y = gaussian_vector(st.n, 2501), gaussian_vector(st.n, 3501)
    M = hm.Matrix(lay, "h2", vals["h2"], task_bytes=2000, spin_limit_us=1, schedule="persistent", **pp)
    aborted = 0
    for _ in range(5):
        out = product(M, x, y)
        try:
            M.check()
        except hm.HMError as e:
            assert e.status == _lib.HM_EDEVICE
            aborted += 1
            continue
        assert np.all(np.isfinite(out))
    print(f"  {aborted} of 5 launches aborted", flush=True)
    M.free()
    M2 = hm.Matrix(lay, "h2", vals["h2"], task_bytes=2000, schedule="persistent", **pp)
    out = product(M2, x, y)
    M2.check()
    ref = stored.product(st, "h2", vals["h2"], 0.75, x, y)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref - y) <= tol
    M2.free()
