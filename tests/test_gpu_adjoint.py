"""GPU parity of the adjoint product y += alpha M^T x (HM_ADJOINT, the
remark after Alg. 3) against the oracle's product of the transposed matrix
stored under the same policy, for single vectors, blocks of right-hand
sides and captured graphs; the adjoint identity <y, M x> = <M^T y, x> on
the GPU's own results; and the error for a matrix uploaded without it."""
import numpy as np
import pytest

from conftest import cached
from oracle import adjoint, stored, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_matrix, gaussian_vector, sphere_points, to_h2, to_uh

pytestmark = pytest.mark.gpu

POLICIES = {
    "f64": (dict(dense="f64", factor="f64", eps=1e-8), 1e-10),
    "fp8": (dict(dense="f32", diag="f64", factor="fp8", coupling="fp8", eps=1e-6), 1e-6),
    "valr6": (dict(dense="valr", diag="valr", factor="valr", eps=1e-6), 1e-6),
}


def case():
    def build():
        import paper_2405_03456_amd as hm
        p = sphere_points(2048, 1001)
        st = trees.build_structure(p)
        lay = hm.Layout(p)
        h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
        return st, lay, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("gpu-adjoint",), build)


def oracle_adjoint(st, fmt, vals, pp, alpha, X, Y):
    tst = adjoint.transpose_structure(st)
    sv = stored.stored_values(tst, fmt, adjoint.transpose_values(fmt, vals), dense=pp["dense"], diag=pp.get("diag"),
                              factor=pp["factor"], coupling=pp.get("coupling"), eps=pp["eps"])
    return stored.product_many(tst, fmt, sv, alpha, X, Y)


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", list(POLICIES))
def test_adjoint_parity(fmt, pol):
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, tol = POLICIES[pol]
    print(f"case adjoint {fmt} {pol}", flush=True)
    n = st.n
    M = hm.Matrix(lay, fmt, vals[fmt], adjoint=True, **pp)
    x, y = gaussian_vector(n, 2701), gaussian_vector(n, 3701)
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, yd, alpha=-0.5, adjoint=True)
    torch.cuda.synchronize()
    ref = oracle_adjoint(st, fmt, vals[fmt], pp, -0.5, x[:, None], y[:, None])[:, 0]
    err = np.linalg.norm(yd.cpu().numpy() - ref) / np.linalg.norm(ref - y)
    print(f"  single vector rel err {err:.3e}", flush=True)
    assert err <= tol
    # a block of 20 right-hand sides, through a captured graph
    X = gaussian_matrix(n, 20, 2702)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda().T
    Yd = torch.zeros((20, n), dtype=torch.float64, device="cuda").T
    g = hm.BatchGraph([M], [Xd], [Yd], adjoint=True)
    g.launch()
    torch.cuda.synchronize()
    R = oracle_adjoint(st, fmt, vals[fmt], pp, 1.0, X, np.zeros((n, 20)))
    e = (np.linalg.norm(Yd.cpu().numpy() - R, axis=0) / np.linalg.norm(R, axis=0)).max()
    print(f"  20 columns worst rel err {e:.3e}", flush=True)
    assert e <= tol
    g.free()
    M.free()


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
def test_adjoint_identity_on_the_gpu(fmt):
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    n = st.n
    M = hm.Matrix(lay, fmt, vals[fmt], adjoint=True, dense="f64", factor="f64", eps=1e-8)
    x, y = gaussian_vector(n, 5), gaussian_vector(n, 6)
    xd, ydv = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    ax = torch.zeros(n, dtype=torch.float64, device="cuda")
    aty = torch.zeros(n, dtype=torch.float64, device="cuda")
    M.mvm(xd, ax)
    M.mvm(ydv, aty, adjoint=True)
    torch.cuda.synchronize()
    lhs, rhs = float(y @ ax.cpu().numpy()), float(aty.cpu().numpy() @ x)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(ax.cpu().numpy()) * np.linalg.norm(y)
    M.free()


def test_adjoint_needs_the_upload_option():
    import torch
    import paper_2405_03456_amd as hm
    from paper_2405_03456_amd import _lib
    st, lay, vals = case()
    M = hm.Matrix(lay, "h", vals["h"], dense="f64", factor="f64", eps=1e-8)
    x = torch.zeros(st.n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(hm.HMError) as ex:
        M.mvm(x, y, adjoint=True)
    assert ex.value.status == _lib.HM_EINVAL
    M.free()
