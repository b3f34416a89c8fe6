"""GPU tests of the two schedules of the H2 downward pass (Alg. 7):
couplings of every level in one launch right after the upward pass
(default), and couplings with the transfers of their level.  Both against
the oracle, under several storage policies and task sizes; the persistent
schedule bitwise equal to the staged one; many right-hand sides."""
import numpy as np
import pytest

from conftest import cached
from oracle import stored, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_matrix, gaussian_vector, sphere_points, to_h2

pytestmark = pytest.mark.gpu

POLICIES = {
    "f64": (dict(dense="f64", factor="f64", eps=1e-8), 1e-10),
    "valr": (dict(dense="valr", diag="valr", factor="valr", eps=1e-6), 1e-6),
    "aflp": (dict(dense="aflp", diag="aflp", factor="aflp", coupling="aflp", eps=1e-6), 1e-6),
}


def case():
    def build():
        import paper_2405_03456_amd as hm
        p = sphere_points(4096, 1201)
        st = trees.build_structure(p)
        lay = hm.Layout(p)
        h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
        return st, lay, to_h2(h, st)
    return cached(("h2-levels",), build)


def product(M, x, y, alpha):
    import torch
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, yd, alpha=alpha)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("pol", list(POLICIES))
@pytest.mark.parametrize("tb", [0, 2000])
def test_h2_level_schedules_parity(pol, tb):
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, tol = POLICIES[pol]
    print(f"case h2 level schedules {pol} task_bytes={tb}", flush=True)
    x, y = gaussian_vector(st.n, 6101), gaussian_vector(st.n, 7101)
    sv = stored.stored_values(st, "h2", vals, dense=pp["dense"], diag=pp.get("diag"), factor=pp["factor"],
                              coupling=pp.get("coupling"), eps=pp["eps"])
    ref = stored.product(st, "h2", sv, 0.5, x, y)
    outs = {}
    for lv in ("coupling_first", "per_level"):
        M = hm.Matrix(lay, "h2", vals, task_bytes=tb, h2_levels=lv, **pp)
        outs[lv] = product(M, x, y, 0.5)
        err = np.linalg.norm(outs[lv] - ref) / np.linalg.norm(ref - y)
        print(f"  {lv}: rel err {err:.3e} (tol {tol:g}), {M.stats()['nlaunch']} launches", flush=True)
        assert err <= tol
        M.free()
    d = np.linalg.norm(outs["coupling_first"] - outs["per_level"]) / np.linalg.norm(ref - y)
    assert d <= tol


@pytest.mark.parametrize("pol", list(POLICIES))
def test_h2_coupling_first_persistent_and_batch(pol):
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, tol = POLICIES[pol]
    print(f"case h2 coupling-first persistent/batch {pol}", flush=True)
    x, y = gaussian_vector(st.n, 6201), gaussian_vector(st.n, 7201)
    Ms = hm.Matrix(lay, "h2", vals, task_bytes=3000, **pp)
    Mp = hm.Matrix(lay, "h2", vals, task_bytes=3000, schedule="persistent", **pp)
    a = product(Ms, x, y, 1.5)
    b = product(Mp, x, y, 1.5)
    Mp.check()
    assert np.array_equal(a, b)
    n, r = st.n, 24
    X, Y = gaussian_matrix(n, r, 6301), gaussian_matrix(n, r, 7301)
    sv = stored.stored_values(st, "h2", vals, dense=pp["dense"], diag=pp.get("diag"), factor=pp["factor"],
                              coupling=pp.get("coupling"), eps=pp["eps"])
    R = stored.product_many(st, "h2", sv, -1.0, X, Y)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda().T
    Yd = torch.from_numpy(np.ascontiguousarray(Y.T)).cuda().T
    Ms.mvm_many(Xd, Yd, alpha=-1.0)
    torch.cuda.synchronize()
    e = (np.linalg.norm(Yd.cpu().numpy() - R, axis=0) / np.linalg.norm(R - Y, axis=0)).max()
    print(f"  batch worst column rel err {e:.3e}", flush=True)
    assert e <= tol
    Ms.free()
    Mp.free()
