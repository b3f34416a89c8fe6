"""GPU parity of the byte-aligned codecs of Sec. 4.1 (FPX rows, AFLP widths)
against the oracle's product of the matrix stored under the same policy:
the adaptive policies (direct compression at eps, VALR over the codec's
widths, Sec. 4.2) and every fixed width, so that each decoder runs; single
vectors with whole and split owners, the persistent schedule (bitwise equal
to the staged one), and blocks of right-hand sides on the matrix cores."""
import numpy as np
import pytest

from conftest import cached
from oracle import codecs, stored, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_matrix, gaussian_vector, sphere_points, to_h2, to_uh

pytestmark = pytest.mark.gpu


def _all(name, eps):
    return dict(dense=name, diag=name, factor=name, coupling=name, eps=eps)


# name -> (storage policy, tolerance of the relative error against the
# oracle's product of the same stored matrix)
POLICIES = {
    "aflp_e6": (_all("aflp", 1e-6), 1e-6),
    "fpx_e6": (_all("fpx", 1e-6), 1e-6),
    "aflp_e8": (_all("aflp", 1e-8), 1e-10),
    "fpx_e8": (_all("fpx", 1e-8), 1e-10),
    "aflp_factor_f64_diag": (dict(dense="aflp", diag="f64", factor="aflp", coupling="aflp", eps=1e-6), 1e-6),
    **{f"aflp{8 * b}": (_all(f"aflp{8 * b}", 1e-6), 1e-6) for b in range(1, 8)},
    **{n: (_all(n, 1e-6), 1e-6) for n in ("fpx24", "fpx40", "fpx48", "fpx56")},
}


def case():
    def build():
        import paper_2405_03456_amd as hm
        p = sphere_points(2048, 1001)
        st = trees.build_structure(p)
        lay = hm.Layout(p)
        h = compress_h(p, KERNEL_LAPLACE, st, 1e-8, method="svd")
        return st, lay, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    return cached(("gpu-codecs",), build)


def stored_case(fmt, pol):
    st, _, vals = case()
    pp, _ = POLICIES[pol]

    def build():
        counts = np.zeros(stored.NCODES, dtype=np.int64)
        sv = stored.stored_values(st, fmt, vals[fmt], dense=pp["dense"], diag=pp.get("diag"), factor=pp["factor"],
                                  coupling=pp.get("coupling"), eps=pp["eps"], counts=counts)
        return sv, counts
    return cached(("gpu-codecs-stored", fmt, pol), build)


def product(M, x, y, alpha):
    import torch
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, yd, alpha=alpha)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", list(POLICIES))
@pytest.mark.parametrize("tb", [0, 2000])
def test_codec_single_vector_parity(fmt, pol, tb):
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, tol = POLICIES[pol]
    print(f"case codec single-vector {fmt} {pol} task_bytes={tb}", flush=True)
    sv, counts = stored_case(fmt, pol)
    M = hm.Matrix(lay, fmt, vals[fmt], task_bytes=tb, **pp)
    s = M.stats()
    # the library stores exactly the oracle's formats
    assert s["entries_per_dtype"] == [int(c) for c in counts[:17]]
    x, y = gaussian_vector(st.n, 4101), gaussian_vector(st.n, 5101)
    out = product(M, x, y, -0.75)
    ref = stored.product(st, fmt, sv, -0.75, x, y)
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref - y)
    print(f"  rel err {err:.3e} (tol {tol:g}); formats "
          f"{ {hm.DTYPE_NAMES[d]: int(c) for d, c in enumerate(counts[:17]) if c} }", flush=True)
    assert err <= tol
    # a second product over the same upload gives the same bits
    assert np.array_equal(product(M, x, y, -0.75), out)
    M.free()


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", ["aflp_e6", "fpx_e8", "aflp24", "fpx40"])
def test_codec_persistent_equals_staged(fmt, pol):
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, _ = POLICIES[pol]
    print(f"case codec persistent vs staged {fmt} {pol}", flush=True)
    x, y = gaussian_vector(st.n, 4201), gaussian_vector(st.n, 5201)
    Mp = hm.Matrix(lay, fmt, vals[fmt], task_bytes=3000, schedule="persistent", **pp)
    Ms = hm.Matrix(lay, fmt, vals[fmt], task_bytes=3000, schedule="staged", **pp)
    a = product(Mp, x, y, 1.25)
    b = product(Ms, x, y, 1.25)
    Mp.check()
    assert np.array_equal(a, b)
    Mp.free()
    Ms.free()


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", ["aflp_e6", "fpx_e6", "aflp_e8", "aflp8", "aflp16", "aflp32", "aflp56",
                                 "fpx24", "fpx48"])
@pytest.mark.parametrize("r", [16, 33])
def test_codec_batch_parity(fmt, pol, r):
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, tol = POLICIES[pol]
    n = st.n
    print(f"case codec batch {fmt} {pol} r={r}", flush=True)
    sv, _ = stored_case(fmt, pol)
    X, Y = gaussian_matrix(n, r, 4300 + r), gaussian_matrix(n, r, 5300 + r)
    ref = stored.product_many(st, fmt, sv, 0.5, X, Y)
    M = hm.Matrix(lay, fmt, vals[fmt], **pp)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda().T
    Yd = torch.from_numpy(np.ascontiguousarray(Y.T)).cuda().T
    M.mvm_many(Xd, Yd, alpha=0.5)
    torch.cuda.synchronize()
    out = Yd.cpu().numpy()
    err = (np.linalg.norm(out - ref, axis=0) / np.linalg.norm(ref - Y, axis=0)).max()
    print(f"  worst column rel err {err:.3e} (tol {tol:g})", flush=True)
    M.free()
    assert err <= tol


def test_codec_adjoint_parity():
    """The adjoint upload stores the transposed blocks under the same codec
    policy (per transposed column: its own scale, one exponent width per
    transposed stored matrix)."""
    import torch
    import paper_2405_03456_amd as hm
    from oracle import adjoint
    st, lay, vals = case()
    pp, tol = POLICIES["aflp_e6"]
    print("case codec adjoint uh aflp_e6", flush=True)
    n = st.n
    M = hm.Matrix(lay, "uh", vals["uh"], adjoint=True, **pp)
    x, y = gaussian_vector(n, 4401), gaussian_vector(n, 5401)
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y.copy()).cuda()
    M.mvm(xd, yd, alpha=2.0, adjoint=True)
    torch.cuda.synchronize()
    tst = adjoint.transpose_structure(st)
    sv = stored.stored_values(tst, "uh", adjoint.transpose_values("uh", vals["uh"]), dense=pp["dense"],
                              diag=pp["diag"], factor=pp["factor"], coupling=pp["coupling"], eps=pp["eps"])
    ref = stored.product(tst, "uh", sv, 2.0, x, y)
    err = np.linalg.norm(yd.cpu().numpy() - ref) / np.linalg.norm(ref - y)
    print(f"  rel err {err:.3e}", flush=True)
    M.free()
    assert err <= tol


def _scaled(vals, fmt, f):
    """The values of every stored matrix times f (a power of two: exact)."""
    import copy
    out = copy.copy(vals)
    for name in ("dense", "W", "coupling"):
        if hasattr(vals, name) and getattr(vals, name) is not None:
            setattr(out, name, [None if a is None else a * f for a in getattr(vals, name)])
    return out


@pytest.mark.parametrize("fmt", ["h", "uh", "h2"])
@pytest.mark.parametrize("pol", ["aflp_e6", "fpx_e6", "aflp_e8", "aflp16", "fpx40"])
@pytest.mark.parametrize("shift", [-90, 90])
def test_codec_extreme_magnitudes(fmt, pol, shift):
    """Matrices scaled by 2^-90 and 2^90 (exactly): AFLP's per-column scale
    exponents and FPX's exponents far from 1; the product stays within the
    tolerance of the oracle's product of the same stored values, and equals
    2^shift times the unscaled product's increment to rounding."""
    import paper_2405_03456_amd as hm
    st, lay, vals = case()
    pp, tol = POLICIES[pol]
    f = 2.0 ** shift
    sv0 = _scaled(vals[fmt], fmt, f)
    print(f"case codec magnitude {fmt} {pol} 2^{shift}", flush=True)
    sv = stored.stored_values(st, fmt, sv0, dense=pp["dense"], diag=pp.get("diag"), factor=pp["factor"],
                              coupling=pp.get("coupling"), eps=pp["eps"])
    M = hm.Matrix(lay, fmt, sv0, **pp)
    x, y = gaussian_vector(st.n, 4501), gaussian_vector(st.n, 5501) * f
    out = product(M, x, y, 1.0)
    ref = stored.product(st, fmt, sv, 1.0, x, y)
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref - y)
    print(f"  rel err {err:.3e} (tol {tol:g})", flush=True)
    assert np.all(np.isfinite(out)) and err <= tol
    M.free()
