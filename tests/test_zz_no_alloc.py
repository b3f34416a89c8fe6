"""hm_mvm_batch_noalloc (callers that cannot allocate): its products equal
hm_mvm_batch's bitwise, on two calls in a row (the second with a smaller
input, so the shared scratch array holds the first call's contents), and a
call whose workspaces exceed the array is refused before anything runs."""
import numpy as np
import pytest

from conftest import cached
from oracle import stored, trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_matrix, sphere_points, to_uh

pytestmark = pytest.mark.gpu


def case():
    def build():
        import paper_2405_03456_amd as hm
        out = {}
        for n, seed, fmt in ((2048, 1001, "h"), (1500, 77, "uh")):
            p = sphere_points(n, seed)
            st = trees.build_structure(p)
            lay = hm.Layout(p)
            h = compress_h(p, KERNEL_LAPLACE, st, 1e-6, method="svd")
            out[fmt] = (st, lay, h if fmt == "h" else to_uh(h, st))
        return out
    return cached(("noalloc",), build)


def blocks(torch, n, r, seed):
    X = gaussian_matrix(n, r, seed)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda().T
    return X, Xd


def test_noalloc_equals_batch_two_calls():
    import torch
    import paper_2405_03456_amd as hm
    c = case()
    pol = dict(dense="f32", factor="f32", eps=1e-6)
    Mh = hm.Matrix(c["h"][1], "h", c["h"][2], **pol)
    Mu = hm.Matrix(c["uh"][1], "uh", c["uh"][2], **pol)
    Mh.tune(40, reps=1)            # builds the many-RHS plans (allocates, outside the no-alloc calls)
    Mu.tune(8, reps=1)
    for call, (M, fmt, r, seed) in enumerate(((Mh, "h", 40, 11), (Mu, "uh", 7, 12))):
        st = c[fmt][0]
        n = st.n
        print(f"case noalloc call {call}: {fmt} n={n} r={r}", flush=True)
        X, Xd = blocks(torch, n, r, seed)
        Y0 = gaussian_matrix(n, r, seed + 100)
        Ya = torch.from_numpy(np.ascontiguousarray(Y0.T)).cuda().T
        Yb = torch.from_numpy(np.ascontiguousarray(Y0.T)).cuda().T
        hm.mvm_batch_noalloc([M], [Xd], [Ya], alpha=-0.5)
        hm.mvm_batch([M], [Xd], [Yb], alpha=-0.5)
        torch.cuda.synchronize()
        A, B = Ya.cpu().numpy(), Yb.cpu().numpy()
        assert np.array_equal(A, B)
        sv = stored.stored_values(st, fmt, c[fmt][2], **pol)
        ref = stored.product_many(st, fmt, sv, -0.5, X, Y0)
        err = (np.linalg.norm(A - ref, axis=0) / np.linalg.norm(ref - Y0, axis=0)).max()
        assert err <= 1e-6, err
    Mh.free()
    Mu.free()


def test_noalloc_refuses_oversized_calls():
    import torch
    import paper_2405_03456_amd as hm
    from paper_2405_03456_amd import _lib
    c = case()
    st, lay, vals = c["h"]
    M = hm.Matrix(lay, "h", vals, dense="f32", factor="f32", eps=1e-6)
    X, Xd = blocks(torch, st.n, 1024, 13)
    Y = torch.zeros((1024, st.n), dtype=torch.float64, device="cuda").T
    with pytest.raises(hm.HMError) as ex:       # plan not built yet
        hm.mvm_batch_noalloc([M], [Xd], [Y])
    assert ex.value.status == _lib.HM_EINVAL
    M.tune(16, reps=1)
    with pytest.raises(hm.HMError) as ex:       # 1024 columns: workspaces beyond the array
        hm.mvm_batch_noalloc([M], [Xd], [Y])
    assert ex.value.status == _lib.HM_EINVAL and "HM_NOALLOC_SCRATCH_BYTES" in str(ex.value)
    torch.cuda.synchronize()
    assert float(Y.abs().max()) == 0.0          # nothing ran
    M.free()
