"""Parity at the full workload sizes, in the launch configuration the
benchmark times (HIP graph replays of rotated copies), over whole output
vectors against the oracle (C/OpenMP product of the same stored values):

* UH n=32768, H n=131072 (FP64 / FP32 / VALR / BF16 storage);
* H2 n=262144, eps 1e-6, with the factors, couplings and transfers in FP64,
  FP32, BF16, FP8 and VALR (FP32 near field, FP64 diagonal near field);
* H n=131072, eps 1e-6, blocks of 8, 32 and 128 right-hand sides with FP32
  and BF16 storage through the tuned many-RHS plan, every column;
* the serving mix: 16 resident H / UH / H2 matrices, n drawn from
  [8192, 131072], Laplace and exp(-r)/r kernels, eps in {1e-4, 1e-6, 1e-8};
  every request bitwise the same alone and in a Poisson mix, and against the
  oracle.

Generated inputs are cached on disk (synth.cache) and shared with the
benchmark on the same machine; the first generation of the H2 n=262144
matrix takes about a minute.
"""
import time

import numpy as np
import pytest

from conftest import cached, say
from oracle import omp, stored, trees
from synth import (KERNEL_EXPR, KERNEL_LAPLACE, cache, compress_h, gaussian_matrix, gaussian_vector,
                   sphere_points, to_h2, to_uh)

pytestmark = pytest.mark.gpu


def workload(fmt, n, seed, eps=1e-6, kernel=KERNEL_LAPLACE):
    """(oracle structure, layout, values); the layout equals the oracle's
    tree bit for bit (checked here before use)."""
    def build():
        import paper_2405_03456_amd as hm
        p = sphere_points(n, seed)
        st = trees.build_structure(p)
        lay = hm.Layout(p)
        e = lay.export()
        assert np.array_equal(e["perm"], st.perm) and np.array_equal(e["blk_tau"], st.blk_tau)
        assert np.array_equal(e["blk_sigma"], st.blk_sigma) and np.array_equal(e["blk_adm"], st.blk_adm)

        def gen():
            say(f"  building {fmt} n={n}: H compression")
            h = compress_h(p, kernel, st, eps, method="auto")
            if fmt != "h":
                say(f"  building {fmt} n={n}: nested bases")
            return h if fmt == "h" else to_uh(h, st) if fmt == "uh" else to_h2(h, st)
        vals = cache.cached(("test-full", fmt, n, seed, eps, kernel), gen)
        say(f"  {fmt} n={n} ready")
        return st, lay, vals
    return cached(("full", fmt, n, seed, eps, kernel), build)


def graph_parity(fmt, n, seed, pol, tol, copies=2):
    import torch
    import paper_2405_03456_amd as hm
    st, lay, vals = workload(fmt, n, seed)
    x = gaussian_vector(n, 2000 + seed % 1000)
    say("  oracle: stored values and product")
    sv = stored.stored_values(st, fmt, vals, dense=pol["dense"], diag=pol.get("diag"), factor=pol["factor"],
                              coupling=pol.get("coupling"), eps=pol["eps"])
    ref = omp.product(st, fmt, sv, 1.0, x, np.zeros(n))
    del sv
    say("  upload and tune")
    Ms = [hm.Matrix(lay, fmt, vals, **pol) for _ in range(copies)]     # rotated copies, as in bench.py
    for M in Ms:
        M.tune_mvm(reps=3)
    xd = torch.from_numpy(x).cuda()
    ys = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in Ms]
    gs = [M.graph(xd, y) for M, y in zip(Ms, ys)]
    for _ in range(3):
        for g in gs:
            g.launch()
    torch.cuda.synchronize()
    for y in ys:
        err = float(np.linalg.norm(y.cpu().numpy() / 3.0 - ref) / np.linalg.norm(ref))
        say(f"  rel err {err:.3e} (tol {tol:g})")
        assert err <= tol
    for g in gs:
        g.free()
    for M in Ms:
        M.free()


CASES = [("uh", 32768, 1002, "f64", dict(dense="f64", factor="f64", eps=1e-6), 1e-10),
         ("uh", 32768, 1002, "f32", dict(dense="f32", factor="f32", eps=1e-6), 1e-6),
         ("uh", 32768, 1002, "valr", dict(dense="valr", diag="valr", factor="valr", eps=1e-6), 1e-6),
         ("h", 131072, 1004, "f64", dict(dense="f64", factor="f64", eps=1e-6), 1e-10),
         ("h", 131072, 1004, "bf16", dict(dense="bf16", factor="bf16", eps=1e-6), 1e-6),
         ("h", 131072, 1004, "valr", dict(dense="valr", diag="valr", factor="valr", eps=1e-6), 1e-6)]


@pytest.mark.parametrize("fmt,n,seed,pname,pol,tol", CASES, ids=[f"{c[0]}{c[1]}-{c[3]}" for c in CASES])
def test_fullsize_graph_parity(fmt, n, seed, pname, pol, tol):
    say(f"case fullsize {fmt} n={n} policy={pname}")
    graph_parity(fmt, n, seed, pol, tol)


# H2 n=262144, eps 1e-6: the benchmark's storage ladder
H2_CASES = [("f64", dict(dense="f64", diag="f64", factor="f64", coupling="f64", eps=1e-6), 1e-10),
            ("f32", dict(dense="f32", diag="f64", factor="f32", coupling="f32", eps=1e-6), 1e-6),
            ("bf16", dict(dense="f32", diag="f64", factor="bf16", coupling="bf16", eps=1e-6), 1e-6),
            ("fp8", dict(dense="f32", diag="f64", factor="fp8", coupling="fp8", eps=1e-6), 1e-6),
            ("valr", dict(dense="valr", diag="valr", factor="valr", coupling="valr", eps=1e-6), 1e-6),
            ("aflp", dict(dense="aflp", diag="aflp", factor="aflp", coupling="aflp", eps=1e-6), 1e-6),
            ("fpx", dict(dense="fpx", diag="fpx", factor="fpx", coupling="fpx", eps=1e-6), 1e-6)]


@pytest.mark.parametrize("pname,pol,tol", H2_CASES, ids=[c[0] for c in H2_CASES])
def test_fullsize_h2_262144(pname, pol, tol):
    say(f"case fullsize h2 n=262144 policy={pname}")
    graph_parity("h2", 262144, 1003, pol, tol, copies=1)


@pytest.mark.parametrize("pname", ["f32", "bf16"])
def test_fullsize_many_rhs_h131072(pname):
    """H n=131072, blocks of 8, 32 and 128 right-hand sides through the tuned
    many-RHS plan in captured batch graphs, every column against the oracle."""
    import torch
    import paper_2405_03456_amd as hm
    n = 131072
    st, lay, vals = workload("h", n, 1004)
    pol = dict(dense=pname, factor=pname, eps=1e-6)
    sv = stored.stored_values(st, "h", vals, dense=pname, factor=pname, eps=1e-6)
    P = omp.Prepared(st, "h", sv)
    M = hm.Matrix(lay, "h", vals, **pol)
    X = gaussian_matrix(n, 128, 2004)
    for r in (8, 32, 128):
        say(f"case fullsize many-rhs h131072 {pname} r={r}")
        M.tune(r, reps=2)
        Xd = torch.from_numpy(np.ascontiguousarray(X[:, :r].T)).cuda().T
        Yd = torch.zeros((r, n), dtype=torch.float64, device="cuda").T
        g = hm.BatchGraph([M], [Xd], [Yd])
        g.launch()
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy()
        worst = 0.0
        for j in range(r):
            ref = P.product(1.0, X[:, j], np.zeros(n))[0]
            worst = max(worst, float(np.linalg.norm(Y[:, j] - ref) / np.linalg.norm(ref)))
        say(f"  worst column rel err {worst:.3e}")
        assert worst <= 1e-6
        g.free()
    M.free()


def serving_mix():
    """The 16 resident matrices of the serving configuration: matrix i has
    format i mod 3, the Laplace kernel for even i else exp(-r)/r,
    eps = (1e-4, 1e-6, 1e-8)[(i // 3) mod 3], VALR storage for eps >= 1e-6
    else FP64, and n drawn uniformly from [8192, 131072]."""
    rng = np.random.default_rng(4200)
    out = []
    for i in range(16):
        n = int(rng.integers(8192, 131073))
        fmt = ("h", "uh", "h2")[i % 3]
        kern = KERNEL_LAPLACE if i % 2 == 0 else KERNEL_EXPR
        eps = (1e-4, 1e-6, 1e-8)[(i // 3) % 3]
        pol = (dict(dense="valr", diag="valr", factor="valr", coupling="valr", eps=eps) if eps >= 1e-6
               else dict(dense="f64", factor="f64", eps=eps))
        out.append((fmt, n, 4100 + i, eps, kern, pol))
    return out


def test_fullsize_serving_mix():
    import paper_2405_03456_amd as hm
    mix = serving_mix()
    Ms, Ps, ns = [], [], []
    t0 = time.perf_counter()
    for fmt, n, seed, eps, kern, pol in mix:
        st, lay, vals = workload(fmt, n, seed, eps, kern)
        sv = stored.stored_values(st, fmt, vals, dense=pol["dense"], diag=pol.get("diag"), factor=pol["factor"],
                                  coupling=pol.get("coupling"), eps=eps)
        Ps.append(omp.Prepared(st, fmt, sv))
        Ms.append(hm.Matrix(lay, fmt, vals, **pol))
        ns.append(n)
        say(f"  matrix {fmt} n={n} eps={eps:g} ready ({time.perf_counter() - t0:.0f}s)")
    S = hm.Server(mem_budget=2 << 30, max_slots=32, max_queue=1000, max_cols=32)
    ids = [S.register(M) for M in Ms]
    rng = np.random.default_rng(4400)
    reqs = [(int(rng.integers(0, 16)), int(rng.integers(1, 33)), float(rng.exponential(0.0003)),
             float(rng.choice([1.0, -0.5]))) for _ in range(48)]
    Xs = [gaussian_matrix(ns[m], r, 7100 + i) for i, (m, r, _, _) in enumerate(reqs)]
    say(f"case serving mix: 16 matrices, {len(reqs)} requests")
    alone = []
    for (m, r, _, a), X in zip(reqs, Xs):
        t, Y = S.submit(ids[m], X, alpha=a)
        S.wait(t)
        alone.append(Y)
    pend = []
    for (m, r, gap, a), X in zip(reqs, Xs):
        time.sleep(gap)
        pend.append(S.submit(ids[m], X, alpha=a))
    mixed = []
    for t, Y in pend:
        S.wait(t)
        mixed.append(Y)
    st = S.stats()
    assert st["max_group_requests"] > 1          # requests really shared launch groups
    worst = 0.0
    for (m, r, _, a), X, Ya, Ym in zip(reqs, Xs, alone, mixed):
        assert np.array_equal(Ya, Ym)            # bitwise alone == in the mix
        tol = 1e-10 if mix[m][3] < 1e-7 else 1e-6
        for j in range(r):
            ref = Ps[m].product(a, X[:, j], np.zeros(ns[m]))[0]
            err = float(np.linalg.norm(Ya[:, j] - ref) / np.linalg.norm(ref))
            worst = max(worst, err / tol)
            assert err <= tol, (m, j, err)
    say(f"  worst error / tolerance {worst:.3e}; server {st}")
    S.close()
    for M in Ms:
        M.free()
