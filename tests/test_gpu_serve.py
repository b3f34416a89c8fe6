"""GPU tests of the request loop: results against the oracle, and each
request bitwise the same alone and in a mix (a seeded Poisson trace over
three resident matrices)."""
import time

import numpy as np
import pytest

from conftest import cached
from oracle import stored, trees
from synth import KERNEL_EXPR, KERNEL_LAPLACE, compress_h, gaussian_matrix, sphere_points, to_h2, to_uh

pytestmark = pytest.mark.gpu

POL = dict(dense="valr", diag="valr", factor="valr", eps=1e-6)


def resident():
    def build():
        import paper_2405_03456_amd as hm
        out = []
        for i, (fmt, n, kern) in enumerate((("h", 2048, KERNEL_LAPLACE), ("uh", 1500, KERNEL_EXPR),
                                            ("h2", 2500, KERNEL_LAPLACE))):
            p = sphere_points(n, 4100 + i)
            st = trees.build_structure(p)
            lay = hm.Layout(p)
            h = compress_h(p, kern, st, 1e-6, method="svd")
            vals = {"h": h, "uh": to_uh(h, st), "h2": to_h2(h, st)}[fmt]
            sv = stored.stored_values(st, fmt, vals, eps=1e-6, dense="valr", diag="valr", factor="valr")
            out.append((fmt, st, lay, vals, sv))
        return out
    return cached(("serve-resident",), build)


def trace(nreq, seed):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(0, 3)), int(rng.integers(1, 33)), float(rng.exponential(0.0005)),
             float(rng.choice([1.0, -0.5]))) for _ in range(nreq)]


def test_serve_parity_and_alone_equals_mix():
    import paper_2405_03456_amd as hm
    mats = resident()
    Ms = [hm.Matrix(lay, fmt, vals, **POL) for fmt, st, lay, vals, sv in mats]
    S = hm.Server(mem_budget=256 << 20, max_slots=16, max_queue=1000, max_cols=64)
    ids = [S.register(M) for M in Ms]
    reqs = trace(40, 4200)
    Xs = [gaussian_matrix(mats[m][1].n, r, 7000 + i) for i, (m, r, _, _) in enumerate(reqs)]
    print(f"case serve trace of {len(reqs)} requests", flush=True)
    # alone: one request at a time
    alone = []
    for (m, r, _, a), X in zip(reqs, Xs):
        t, Y = S.submit(ids[m], X, alpha=a)
        S.wait(t)
        alone.append(Y)
    # mix: Poisson arrivals while earlier requests run
    pend = []
    for (m, r, gap, a), X in zip(reqs, Xs):
        time.sleep(gap)
        pend.append(S.submit(ids[m], X, alpha=a))
    stats = [S.wait(t) for t, _ in pend]
    assert max(s["group_requests"] for s in stats) > 1          # batching happened
    for i, ((t, Y), Ya) in enumerate(zip(pend, alone)):
        assert np.array_equal(Y, Ya), i                         # bitwise alone == mix
    # parity of every result against the oracle on the same stored values
    worst = 0.0
    for (m, r, _, a), X, Y in zip(reqs, Xs, alone):
        fmt, st, lay, vals, sv = mats[m]
        ref = stored.product_many(st, fmt, sv, a, X, np.zeros_like(X))
        err = np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)
        worst = max(worst, float(err.max()))
    print(f"  worst column rel err {worst:.3e}", flush=True)
    assert worst <= 1e-6
    s = S.stats()
    assert s["completed"] == 2 * len(reqs)
    S.close()
    for M in Ms:
        M.free()


def test_serve_memory_admission_on_device():
    """A budget that holds one 32-column block of the largest matrix at a
    time still completes a burst, never exceeding the budget."""
    import paper_2405_03456_amd as hm
    mats = resident()
    Ms = [hm.Matrix(lay, fmt, vals, **POL) for fmt, st, lay, vals, sv in mats]
    budget = 2 * 2500 * 32 * 8 + 4096
    S = hm.Server(mem_budget=budget, max_slots=8, max_queue=100, max_cols=32)
    ids = [S.register(M) for M in Ms]
    pend = [S.submit(ids[i % 3], gaussian_matrix(mats[i % 3][1].n, 16, 50 + i)) for i in range(12)]
    for t, _ in pend:
        S.wait(t)
    s = S.stats()
    assert s["peak_arena_bytes"] <= budget and s["completed"] == 12
    S.close()
    for M in Ms:
        M.free()
