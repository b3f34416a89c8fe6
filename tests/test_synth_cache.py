"""The on-disk input cache returns exactly the generated inputs (every
array bit for bit, None entries kept), and is keyed by its arguments."""
import numpy as np

from oracle import trees
from synth import KERNEL_LAPLACE, cache, compress_h, sphere_points, to_h2, to_uh


def _same(a, b):
    if a is None or b is None:
        return a is None and b is None
    a, b = np.asarray(a), np.asarray(b)
    return a.shape == b.shape and a.dtype == b.dtype and np.array_equal(a, b)


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("HM_INPUT_CACHE", str(tmp_path))
    p = sphere_points(700, 9)
    st = trees.build_structure(p)
    h = compress_h(p, KERNEL_LAPLACE, st, 1e-6, method="svd")
    vals = (h, to_uh(h, st), to_h2(h, st), p)
    calls = []

    def build():
        calls.append(1)
        return vals
    first = cache.cached(("unit", 700), build)
    again = cache.cached(("unit", 700), build)
    assert len(calls) == 1 and first is vals
    for a, b in zip(vals[:3], again[:3]):
        assert type(a) is type(b)
        for f in a.__dataclass_fields__:
            va, vb = getattr(a, f), getattr(b, f)
            if isinstance(va, list):
                assert len(va) == len(vb) and all(_same(x, y) for x, y in zip(va, vb)), f
                assert all(y is None or y.flags.f_contiguous for y in vb if isinstance(y, np.ndarray))
            elif isinstance(va, np.ndarray):
                assert _same(va, vb), f
            else:
                assert va == vb, f
    assert _same(vals[3], again[3])
    assert cache.load(("unit", 701)) is None
    monkeypatch.setenv("HM_INPUT_CACHE", "off")
    assert cache.load(("unit", 700)) is None
