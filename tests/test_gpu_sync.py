"""GPU parity of the synchronisation variants (Sec. 3.1: atomic updates and
thread-local copies, beside the default row ownership): every format and
two storage policies against the oracle, graph replays included (the
private copies are cleared by each product's final launch), and the
persistent schedule refusing them."""
import numpy as np
import pytest

from conftest import cached
from oracle import stored, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_vector, sphere_points, to_h2, to_uh

pytestmark = pytest.mark.gpu


def case():
    def build():
        import paper_2405_03456_amd as hm
        p = sphere_points(2048, 1001)
        st = trees.build_structure(p)
        lay = hm.Layout(p)
        h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
        return st, lay, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("gpu-sync",), build)


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", ["f64", "valr6"])
@pytest.mark.parametrize("sync", ["atomic", "private"])
@pytest.mark.parametrize("tb", [0, 2000])
def test_sync_variant_parity(fmt, pol, sync, tb):
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, tol = ((dict(dense="f64", factor="f64", eps=1e-8), 1e-10) if pol == "f64"
               else (dict(dense="valr", diag="valr", factor="valr", eps=1e-6), 1e-6))
    print(f"case sync {sync} {fmt} {pol} task_bytes={tb}", flush=True)
    n = st.n
    M = hm.Matrix(lay, fmt, vals[fmt], sync=sync, task_bytes=tb, **pp)
    x, y = gaussian_vector(n, 2801), gaussian_vector(n, 3801)
    sv = stored.stored_values(st, fmt, vals[fmt], dense=pp["dense"], diag=pp.get("diag"), factor=pp["factor"],
                              eps=pp["eps"])
    ref = stored.product(st, fmt, sv, 0.5, x, y)
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, yd, alpha=0.5)
    torch.cuda.synchronize()
    err = np.linalg.norm(yd.cpu().numpy() - ref) / np.linalg.norm(ref - y)
    assert err <= tol, err
    g = M.graph(xd, yd, alpha=0.5)
    for _ in range(3):
        yd.copy_(torch.from_numpy(y))
        g.launch()
        torch.cuda.synchronize()
        err = np.linalg.norm(yd.cpu().numpy() - ref) / np.linalg.norm(ref - y)
        assert err <= tol, err
    g.free()
    M.free()


def test_sync_variants_need_the_staged_schedule():
    import paper_2405_03456_amd as hm
    from paper_2405_03456_amd import _lib
    st, lay, vals = case()
    with pytest.raises(hm.HMError) as ex:
        hm.Matrix(lay, "h", vals["h"], sync="atomic", schedule="persistent")
    assert ex.value.status == _lib.HM_EINVAL
