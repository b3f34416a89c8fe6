"""GPU parity on the BLR and HODLR partitions: the library's layout equals
the oracle's, and H / UH / H^2 products with float64 and VALR storage equal
the oracle's product of the same stored values (1e-10 with float64
accumulation, 1e-6 with float32)."""
import numpy as np
import pytest

from conftest import cached
from oracle import stored, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_vector, sphere_points, to_h2, to_uh

pytestmark = pytest.mark.gpu


def case(kind):
    def build():
        import paper_2405_03456_amd as hm
        p = sphere_points(2048, 1001)
        st = trees.build_structure(p, kind=kind)
        lay = hm.Layout(p, partition=kind)
        e = lay.export()
        for k in ("perm", "begin", "end", "blk_tau", "blk_sigma", "blk_adm"):
            assert np.array_equal(e[k], getattr(st, k)), k
        h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
        return st, lay, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("gpu-partition", kind), build)


@pytest.mark.parametrize("kind", ["hodlr", "blr"])
@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", ["f64", "valr6"])
def test_partition_parity(kind, fmt, pol):
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case(kind)
    pp, tol = ((dict(dense="f64", factor="f64", eps=1e-8), 1e-10) if pol == "f64"
               else (dict(dense="valr", diag="valr", factor="valr", eps=1e-6), 1e-6))
    print(f"case partition {kind} {fmt} {pol}", flush=True)
    x, y = gaussian_vector(st.n, 2601), gaussian_vector(st.n, 3601)
    M = hm.Matrix(lay, fmt, vals[fmt], **pp)
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, yd, alpha=-0.5)
    torch.cuda.synchronize()
    out = yd.cpu().numpy()
    sv = stored.stored_values(st, fmt, vals[fmt], dense=pp["dense"], diag=pp.get("diag"), factor=pp["factor"],
                              eps=pp["eps"])
    ref = stored.product(st, fmt, sv, -0.5, x, y)
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref - y)
    print(f"  rel err {err:.3e}", flush=True)
    assert err <= tol
    M.free()
