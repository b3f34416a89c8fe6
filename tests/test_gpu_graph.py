"""hipGraph replay of a product equals the eager product, bitwise, on every
replay, with unrelated eager work and synchronisations between replays."""
import numpy as np
import pytest

from conftest import cached
from oracle import trees
from synth import KERNEL_LAPLACE, compress_h, gaussian_vector, sphere_points, to_h2, to_uh

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fmt,pol", [("h", "f64"), ("uh", "f32"), ("h2", "bf16")])
def test_graph_replays_match_eager(fmt, pol):
    import torch
    import paper_2405_03456_amd as hm
    assert torch.cuda.is_available()
    n = 3000

    def build():
        p = sphere_points(n, 4242)
        st = trees.build_structure(p)
        h = compress_h(p, KERNEL_LAPLACE, st, 1e-6, method="svd")
        return p, {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}
    p, vals = cached(("graph", n), build)
    lay = hm.Layout(p)
    kw = {"f64": dict(factor="f64", dense="f64", eps=1e-8),
          "f32": dict(factor="f32", dense="f32", eps=1e-6),
          "bf16": dict(factor="bf16", dense="f32", diag="f64", coupling="f32", eps=1e-6)}[pol]
    M = hm.Matrix(lay, fmt, vals[fmt], **kw)
    x = torch.from_numpy(gaussian_vector(n, 1)).cuda()
    ya = torch.from_numpy(gaussian_vector(n, 2)).cuda()
    yb = ya.clone()
    g = M.graph(x, ya, alpha=0.75)
    for rep in range(4):
        g.launch()
        M.mvm(x, yb, alpha=0.75)
        torch.cuda.synchronize()
        assert torch.equal(ya, yb), f"replay {rep} differs from eager"
        z = torch.randn(257, 257, device="cuda", dtype=torch.float64)   # unrelated work
        (z @ z).sum().item()
        torch.cuda.synchronize()
    g.free()
    M.free()
