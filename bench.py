"""Benchmark: hierarchical-matrix product y += A x on one MI355X.

Default workload: H^2 matrix, n = 262144 points uniform on the unit sphere,
Laplace kernel 1/(4 pi r) (zero diagonal), leaf size 64, eta = 2, eps = 1e-6,
nested bases with transfer matrices, one right-hand side x ~ N(0,1).  The
headline (`value`) is the plain FP64 GPU product; beside it the storage
ladder of compressed formats (FP32 / BF16 / FP8 factors, couplings and
transfers with per-column scales, VALR per column, FP64 diagonal near
field), one variant with the whole near field in FP64, and as extra keys the
uniform-H n=32768 FP64 / FP32 product and the H n=2048 correctness case.

A step is one full product (every phase of the format), replayed from a
captured HIP graph.  Inputs are resident in HBM before timing; matrices
smaller than the timed working set target are uploaded several times and
used in turn, so the numbers are HBM numbers, not Infinity Cache numbers.
Each replay is bracketed by HIP events: ms_per_step is the median, with
p10/p90 beside it and the wall-clock mean of the same loop.  GB/s counts the
method's bytes (every stored entry once at its element size, per-column
scales of FP16/FP8 columns, x, y and the coefficient vectors); tile padding
and plan metadata are reported separately as overhead.

Printed: one JSON line with `value` = FP64 GB/s, matvecs/s, the compressed
legs with their measured errors, a roofline object for the dominant kernel
(HIP-event timed inside the timed region), and the CPU oracle (C/OpenMP,
same product) timed on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-MVM achieved HBM GB/s + matvecs/s vs plain FP64 GPU at stated rel. error"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (format, n, eps, point seed, x seed, description)
    "h2_262144": ("h2", 262144, 1e-6, 1003, 2003,
                  "H2-matrix n=262144 sphere points, Laplace 1/(4 pi r), leaf 64, eta 2, eps 1e-6, 1 RHS"),
    "uh32768": ("uh", 32768, 1e-6, 1002, 2002,
                "UH-matrix n=32768 sphere points, Laplace 1/(4 pi r), leaf 64, eta 2, eps 1e-6, 1 RHS"),
    "h131072": ("h", 131072, 1e-6, 1004, 2004,
                "H-matrix n=131072 sphere points, Laplace 1/(4 pi r), leaf 64, eta 2, eps 1e-6, 1 RHS"),
    "h2048": ("h", 2048, 1e-8, 1001, 2001,
              "H-matrix n=2048 sphere points, Laplace 1/(4 pi r), leaf 64, eta 2, eps 1e-8, 1 RHS"),
}

# storage policies of the single-vector legs
POLICIES = {
    "f64": dict(dense="f64", diag="f64", factor="f64", coupling="f64"),
    # compressed: factors / bases, couplings and transfers in the named format;
    # near-field dense leaves FP32 (direct compression at eps 1e-6, Table 1),
    # diagonal near field FP64
    "f32": dict(dense="f32", diag="f64", factor="f32", coupling="f32"),
    "bf16": dict(dense="f32", diag="f64", factor="bf16", coupling="bf16"),
    "fp8": dict(dense="f32", diag="f64", factor="fp8", coupling="fp8"),
    "valr": dict(dense="valr", diag="valr", factor="valr", coupling="valr"),
    # the whole near field in FP64 (the Amdahl cap of compressing only the far field)
    "fp8_nearfield_f64": dict(dense="f64", diag="f64", factor="fp8", coupling="fp8"),
    # uniform FP32 storage of every block (the UH config's FP32 variant)
    "f32_all": dict(dense="f32", diag="f32", factor="f32", coupling="f32"),
    # the paper's own byte-aligned codecs (Sec. 4.1-4.2) for every class:
    # direct compression of dense, coupling and transfer matrices at eps,
    # VALR over the codec's widths for the cluster bases
    "aflp": dict(dense="aflp", diag="aflp", factor="aflp", coupling="aflp"),
    "fpx": dict(dense="fpx", diag="fpx", factor="fpx", coupling="fpx"),
    # synchronisation variants of Sec. 3.1 (FP64 storage): atomic updates of
    # shared rows, and thread-local (here: eight private) copies of y
    "f64_sync_atomic": dict(dense="f64", diag="f64", factor="f64", coupling="f64", sync="atomic"),
    "f64_sync_private": dict(dense="f64", diag="f64", factor="f64", coupling="f64", sync="private"),
    # H2 downward pass with each level's couplings in that level's launch
    # (the default runs every level's couplings in one launch first)
    "f64_per_level": dict(dense="f64", diag="f64", factor="f64", coupling="f64", h2_levels="per_level"),
}
DEFAULT_LEGS = {"h2": "f64,f32,bf16,fp8,valr,aflp,fpx,fp8_nearfield_f64,f64_sync_atomic,f64_sync_private,"
                      "f64_per_level",
                "uh": "f64,f32_all,valr,aflp,fpx", "h": "f64,f32_all,valr,aflp,fpx"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def structure_from_layout(lay):
    from synth import Structure
    e = lay.export()
    return Structure(e["n"], e["perm"], e["begin"], e["end"], e["level"], e["parent"], e["son0"],
                     e["son1"], e["blk_tau"], e["blk_sigma"], e["blk_adm"])


def make_values(fmt, points, st, eps, kernel=0):
    from synth import compress_h, to_h2, to_uh
    h = compress_h(points, kernel, st, eps, method="auto")
    if fmt == "h":
        return h
    if fmt == "uh":
        return to_uh(h, st)
    return to_h2(h, st)


def workload_inputs(hm, name):
    """(layout, structure, values, points) of a workload, generated once per
    machine (synth.cache)."""
    from synth import cache, sphere_points
    fmt, n, eps, pseed, _, _ = WORKLOADS[name]
    points = sphere_points(n, pseed)
    lay = hm.Layout(points)
    st = structure_from_layout(lay)

    def build():
        return make_values(fmt, points, st, eps)
    vals = cache.cached(("bench", name, fmt, n, eps, pseed), build)
    return lay, st, vals, points


def run_variant(hm, torch, lay, fmt, vals, eps, pol, steps, warmup, x, target):
    """Upload rotated copies, replay `steps` captured products with a HIP
    event pair around each replay, then `steps` eager products with
    per-stage HIP events (the phases of the overlapped schedule), then
    `steps` eager products of one more upload whose dense stage starts after
    the whole chain, uncapped, so that it runs alone at its full launch width
    (the per-kernel roofline: the last launches of that kernel, which a
    kernel trace of the same run reports too)."""
    mats = [hm.Matrix(lay, fmt, vals, eps=eps, **pol)]
    s0 = mats[0].stats()
    stored = s0["bytes_dense"] + s0["bytes_factors"] + s0["bytes_coupling"] + s0["bytes_transfer"]
    ncopies = int(min(8, max(1, math.ceil(target / max(stored, 1)))))
    for _ in range(ncopies - 1):
        mats.append(hm.Matrix(lay, fmt, vals, eps=eps, **pol))
    # fork point of the dense stage, timed per matrix (hm_tune_mvm) before capture
    tuned = [m.tune_mvm(reps=10) for m in mats]
    y = torch.zeros_like(x)
    graphs = [m.graph(x, y) for m in mats]
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        graphs[i % ncopies].launch(stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        graphs[i % ncopies].launch(stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = np.array([a.elapsed_time(b) for a, b in ev])      # ms per replay
    # eager products with per-stage event timing
    for m in mats:
        m.timing()
    torch.cuda.synchronize()
    for i in range(steps):
        mats[i % ncopies].mvm(x, y, timing=True)
    torch.cuda.synchronize()
    def collect():
        out = []
        for m in mats:
            for i, ph in enumerate(m.timing()):
                if len(out) <= i:
                    out.append(dict(ph))
                else:
                    out[i]["ms_total"] += ph["ms_total"]
                    out[i]["launches"] += ph["launches"]
        return out
    phases = collect()
    # one more product from a clean y for the accuracy check
    yv = torch.zeros_like(x)
    mats[0].mvm(x, yv)
    torch.cuda.synchronize()
    y_out = yv.cpu().numpy()
    # the dense stage on its own, at its full launch width: one more upload
    # with the fork point after every chain stage and no workgroup cap (the
    # tuned schedule may cap the stage to leave room for the chain); the
    # products are bitwise the same
    nchain = sum(1 for p in phases if p["ntasks"] > 0 and p["name"] != "dense")
    alone = None
    if any(p["name"] == "dense" and p["ntasks"] > 0 for p in phases):
        Ma = hm.Matrix(lay, fmt, vals, eps=eps, fork_after=nchain, **pol)
        Ma.timing()
        for i in range(steps):
            Ma.mvm(x, y, timing=True)
        torch.cuda.synchronize()
        alone = Ma.timing()
        Ma.free()
    for g in graphs:
        g.free()
    for m in mats:
        m.free()
    return dict(stats=s0, ncopies=ncopies, times=times, wall=wall, phases=phases, alone=alone, y=y_out,
                fork_after=[t["fork_after"] for t in tuned],
                dense_split=[[t["fork2"], t["dense_split"]] if t["dense_split"] else None for t in tuned],
                dense_grid=[t["dense_grid"] for t in tuned])


def summarize(res, steps):
    s = res["stats"]
    t = res["times"]
    ms = float(np.median(t))
    mb = float(s["method_bytes"])
    gbs = mb / (ms * 1e-3) / 1e9
    with_tasks = [p for p in res["phases"] if p["ntasks"] > 0 and p["launches"] > 0]
    dom = max(with_tasks, key=lambda p: p["ms_total"]) if with_tasks else None
    roof = None
    if dom and dom["launches"]:
        over_ms = dom["ms_total"] / dom["launches"]
        avg_ms, how = over_ms, "overlapped schedule"
        if dom["name"] == "dense" and res.get("alone"):
            a = [p for p in res["alone"] if p["name"] == "dense" and p["launches"] > 0]
            if a:
                avg_ms, how = a[0]["ms_total"] / a[0]["launches"], "dense stage alone, after the chain, uncapped"
        ach = dom["method_bytes"] / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": f"k_owner_tasks[{dom['name']}]", "avg_launch_us": round(avg_ms * 1e3, 2),
                "launch_timing": how,
                "overlapped_avg_launch_us": round(over_ms * 1e3, 2),
                "bytes_per_launch": int(dom["method_bytes"]),
                "bytes_per_launch_with_padding": int(dom["algorithmic_bytes"])}
    return dict(ms_per_step=ms, p10_ms=float(np.percentile(t, 10)), p90_ms=float(np.percentile(t, 90)),
                wall_ms_per_step=res["wall"] * 1e3 / steps, gbs=gbs, matvecs_per_s=1e3 / ms, roofline=roof,
                method_bytes=mb, overhead_bytes=float(s["algorithmic_bytes"]) - mb,
                copies=res["ncopies"], fork_after=res["fork_after"], dense_split=res["dense_split"],
                dense_grid=res["dense_grid"],
                phases=[{"name": p["name"], "ntasks": p["ntasks"],
                         "us_avg": round(p["ms_total"] * 1e3 / max(p["launches"], 1), 2),
                         "GBs": (round(p["method_bytes"] / (p["ms_total"] / p["launches"]) / 1e6, 1)
                                 if p["launches"] and p["ms_total"] > 0 else None)} for p in res["phases"]])


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("hm_runtime.hip", "hm_device.h", "hm_stream.h", "hm_plan.h", "hm_pack.cpp", "hm_pack.h",
              "hm_quant.cpp", "hm_tasks_a32_lo.hip", "hm_tasks_a32_hi.hip", "hm_tasks_a64_lo.hip",
              "hm_tasks_a64_hi.hip"):
        with open(os.path.join(ROOT, "paper_2405_03456_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, policy, kernel):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary (FETCH_SIZE/WRITE_SIZE scaled by a copy-kernel calibration), or
    None if there is none or the kernel sources changed since."""
    import glob
    cur = kernel_sources_sha()
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        with open(path) as f:
            for line in f:
                if line.startswith("traffic_json:"):
                    t = json.loads(line.split(":", 1)[1])
                    if (t["workload"] == workload and t["policy"] == policy and t.get("kernel") == kernel
                            and t["source_sha"] == cur):
                        return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0
    return None


def cpu_baseline(fmt, st, vals, x, mb, reps=5):
    """The oracle's C/OpenMP product (same stored FP64 values, same
    definition) timed on every core this process may use and on one core:
    median of `reps` products each, plus a host triad probe."""
    from oracle import omp
    P = omp.Prepared(st, fmt, vals)
    y0 = np.zeros(len(x))
    out = {}
    for label, threads in (("all_cores", 0), ("one_core", 1)):
        ts, used = [], 1
        P.product(1.0, x, y0, threads)                       # warm-up
        for _ in range(reps):
            t0 = time.perf_counter()
            _, used = P.product(1.0, x, y0, threads)
            ts.append(time.perf_counter() - t0)
        dt = float(np.median(ts))
        out[label] = {"seconds": dt, "GBs": mb / dt / 1e9, "matvecs_per_s": 1.0 / dt, "threads": used}
    triad, tused = omp.triad_gbs()
    out["triad_GBs"] = triad
    out["triad_threads"] = tused
    return out


def parity(fmt, st, vals, pol, eps, x, y_gpu, points, rows):
    """Relative errors of a GPU result: against the oracle's product of the
    same stored values (C/OpenMP oracle on the dequantised values), and
    against the dense kernel product on sampled rows (the stated accuracy)."""
    from oracle import dense as odense
    from oracle import omp, stored
    y0 = np.zeros(len(x))
    sv = vals if pol["factor"] == "f64" and pol["dense"] == "f64" and pol["coupling"] == "f64" else \
        stored.stored_values(st, fmt, vals, dense=pol["dense"], diag=pol.get("diag"), factor=pol["factor"],
                             coupling=pol["coupling"], eps=eps)
    ref = omp.product(st, fmt, sv, 1.0, x, y0)
    del sv
    yd = odense.dense_product(0, points, 1.0, x, y0, rows=rows)
    return {"vs_oracle_same_storage": float(np.linalg.norm(y_gpu - ref) / np.linalg.norm(ref)),
            "vs_dense_sampled_rows": float(np.linalg.norm(y_gpu[rows] - yd[rows]) / np.linalg.norm(yd[rows])),
            "oracle_vs_dense_sampled_rows": float(np.linalg.norm(ref[rows] - yd[rows]) / np.linalg.norm(yd[rows]))}


def single_vector(args, hm, torch, name, legs, with_cpu, with_parity):
    """All storage legs of one single-vector workload."""
    from synth import gaussian_vector
    fmt, n, eps, pseed, xseed, desc = WORKLOADS[name]
    t0 = time.perf_counter()
    lay, st, vals, points = workload_inputs(hm, name)
    log(f"[bench] {name}: inputs ready in {time.perf_counter() - t0:.1f}s (blocks={st.nblocks})")
    x_np = gaussian_vector(n, xseed)
    x = torch.from_numpy(x_np).cuda()
    rows = np.arange(0, n, max(1, n // 2048))
    out = {"workload": desc, "format": fmt, "n": n, "eps": eps, "legs": {}}
    base = None
    for leg in legs:
        pol = POLICIES[leg]
        r = run_variant(hm, torch, lay, fmt, vals, eps, pol, args.steps, args.warmup, x, args.copies_bytes)
        sm = summarize(r, args.steps)
        row = {"GBs": round(sm["gbs"], 1), "matvecs_per_s": round(sm["matvecs_per_s"], 1),
               "ms_per_step": round(sm["ms_per_step"], 5), "p10_ms": round(sm["p10_ms"], 5),
               "p90_ms": round(sm["p90_ms"], 5), "wall_ms_per_step": round(sm["wall_ms_per_step"], 5),
               "method_bytes_per_matvec": int(sm["method_bytes"]),
               "overhead_bytes_per_matvec": int(sm["overhead_bytes"]),
               "bytes_per_dtype": r["stats"]["bytes_per_dtype"], "entries_per_dtype": r["stats"]["entries_per_dtype"],
               "fork_after": sm["fork_after"], "dense_split": sm["dense_split"], "dense_grid": sm["dense_grid"],
               "copies": sm["copies"],
               "roofline": sm["roofline"],
               "policy": pol}
        if base is None:
            base = sm
        row["speedup_vs_f64"] = round(base["ms_per_step"] / sm["ms_per_step"], 3)
        if with_parity:
            row["rel_err"] = parity(fmt, st, vals, pol, eps, x_np, r["y"], points, rows)
        out["legs"][leg] = row
        out.setdefault("phases", {})[leg] = sm["phases"]
        log(f"[bench] {name} {leg}: {sm['ms_per_step'] * 1e3:.1f} us/step (p10 {sm['p10_ms'] * 1e3:.1f}, "
            f"p90 {sm['p90_ms'] * 1e3:.1f}), {sm['gbs']:.0f} GB/s, copies={r['ncopies']}, "
            f"rel_err={row.get('rel_err')}")
    if with_cpu:
        mb = out["legs"][legs[0]]["method_bytes_per_matvec"]
        cb = cpu_baseline(fmt, st, vals, x_np, mb)
        out["cpu"] = cb
        log(f"[bench] {name} cpu oracle: {json.dumps(cb)}")
    return out


MFMA_PEAK_TFS = {True: 78.6, False: 157.3}     # float64 / float32 dense matrix-core peaks

MANY_POLICIES = {
    "f64": dict(dense="f64", factor="f64", coupling="f64"),
    "f32": dict(dense="f32", factor="f32", coupling="f32"),
    "bf16": dict(dense="bf16", factor="bf16", coupling="bf16"),
    "valr": dict(dense="valr", diag="valr", factor="valr", coupling="valr"),
    "aflp": dict(dense="aflp", diag="aflp", factor="aflp", coupling="aflp"),
    "fpx": dict(dense="fpx", diag="fpx", factor="fpx", coupling="fpx"),
}
# bytes of one stored value per dtype code (include/hm.h; code 5 is a policy)
DTYPE_BYTES = (8, 4, 2, 2, 1, 0, 3, 5, 6, 7, 1, 2, 3, 4, 5, 6, 7)


def many_rhs(args, hm, torch, lay, fmt, vals, eps, n, points, st, desc):
    """Blocks of r right-hand sides through hm_mvm_batch (graph-replayed),
    per storage policy; per-kernel MFMA roofline from event-timed launches."""
    from synth import gaussian_matrix
    widths = [int(v) for v in args.nrhs.split(",")]
    pols = args.policies.split(",")
    rows = []
    base_ms = None
    Xall = gaussian_matrix(n, max(widths), 2004)
    for pname in pols:
        M = hm.Matrix(lay, fmt, vals, eps=eps, **MANY_POLICIES[pname])
        ref = None
        if not args.no_parity:
            from oracle import omp as oomp
            from oracle import stored as ostored
            sv = ostored.stored_values(st, fmt, vals, eps=eps, **MANY_POLICIES[pname])
            ref = oomp.product(st, fmt, sv, 1.0, Xall[:, 0], np.zeros(n))
            del sv
        s = M.stats()
        entries = sum(s["entries_per_dtype"])
        stored_b = float(sum(c * DTYPE_BYTES[d] for d, c in enumerate(s["entries_per_dtype"])))
        vec_b = float(s["method_bytes"]) - stored_b        # x, y, coefficients (+ FP16/FP8 column scales)
        acc64 = s["accum"] == hm.HM_ACC_F64
        for r in widths:
            X = torch.from_numpy(np.ascontiguousarray(Xall[:, :r].T)).cuda().T
            Y = torch.zeros((r, n), dtype=torch.float64, device="cuda").T
            tuned = None
            if r == 1:
                X, Y = X[:, 0].contiguous(), Y[:, 0].contiguous()
            elif not args.no_tune:
                tuned = M.tune(r, reps=3)
            g = hm.BatchGraph([M], [X], [Y])
            for _ in range(args.warmup):
                g.launch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                g.launch()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / args.steps
            g.free()
            M.timing()
            for _ in range(max(3, args.steps // 5)):
                hm.mvm_batch([M], [X], [Y], timing=True)
            torch.cuda.synchronize()
            ph = [p for p in M.timing() if p["launches"] > 0]
            dom = max(ph, key=lambda p: p["ms_total"] / p["launches"])
            us = dom["ms_total"] * 1e3 / dom["launches"]
            flops = 2.0 * dom["data_entries"] * r
            gbs_dom = dom["data_bytes"] / (us * 1e-6) / 1e9
            alg = stored_b + vec_b * r                        # the method's bytes for r columns
            row = {"policy": pname, "nrhs": r, "ms_per_step": round(ms, 4), "tuned": tuned,
                   "columns_per_s": round(r * 1e3 / ms, 1), "GBs": round(alg / (ms * 1e-3) / 1e9, 1),
                   "TFLOPs": round(2.0 * entries * r / (ms * 1e-3) / 1e12, 2),
                   "dominant": {"phase": dom["name"], "avg_launch_us": round(us, 2),
                                "data_GBs": round(gbs_dom, 1),
                                "TFLOPs": round(flops / (us * 1e-6) / 1e12, 2),
                                "mfma_peak_TFLOPs": None if r == 1 else MFMA_PEAK_TFS[acc64 or pname == "f64"]}}
            if pname == "f64" and r == 1:
                base_ms = ms
            if base_ms is not None:
                row["speedup_vs_f64_single_per_column"] = round(base_ms * r / ms, 2)
            # accuracy of the first column against the oracle on the same stored values
            if ref is not None:
                got = (Y if r == 1 else Y[:, 0]).cpu().numpy() / (args.warmup + args.steps + max(3, args.steps // 5))
                row["rel_err_col0_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            row["phases"] = [{"name": p["name"], "ntasks": p["ntasks"],
                              "us": round(p["ms_total"] * 1e3 / p["launches"], 1),
                              "TFLOPs": round(2.0 * p["data_entries"] * r / (p["ms_total"] * 1e-3 / p["launches"])
                                              / 1e12, 2)} for p in ph]
            log(f"[bench] {json.dumps(row)}")
            rows.append(row)
            del X, Y
        M.free()
    best = max(rows, key=lambda r: r["columns_per_s"])
    out = {"metric": "H-MVM many-RHS matvec columns/s (hm_mvm_batch)", "value": best["columns_per_s"],
           "unit": "columns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": best["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic (seeded sphere points, Laplace kernel, ACA-compressed)",
           "config": {"workload": desc, "format": fmt, "n": n, "eps": eps}, "runs": rows}
    print(json.dumps(out), flush=True)


def serve_mix(args, hm, torch):
    """Serving mix: resident H/UH/H2 matrices, Poisson arrivals of 1..32
    column requests at fractions of the measured capacity."""
    from synth import (KERNEL_EXPR, KERNEL_LAPLACE, compress_h, gaussian_matrix, sphere_points, to_h2, to_uh)
    rng = np.random.default_rng(4200)
    nm = args.serve_matrices
    eps_of = [1e-4, 1e-6, 1e-8]
    mats, info = [], []
    t0 = time.perf_counter()
    for i in range(nm):
        n = int(rng.integers(8192, args.serve_nmax + 1))
        fmt = ("h", "uh", "h2")[i % 3]
        kern = KERNEL_LAPLACE if i % 2 == 0 else KERNEL_EXPR
        eps = eps_of[(i // 3) % 3]
        p = sphere_points(n, 4100 + i)
        lay = hm.Layout(p)
        st = structure_from_layout(lay)
        h = compress_h(p, kern, st, eps, method="auto")
        vals = h if fmt == "h" else to_uh(h, st) if fmt == "uh" else to_h2(h, st)
        pol = dict(dense="valr", diag="valr", factor="valr") if eps >= 1e-6 else dict(dense="f64", factor="f64")
        M = hm.Matrix(lay, fmt, vals, eps=eps, **pol)
        s = M.stats()
        mats.append(M)
        info.append(dict(n=n, fmt=fmt, eps=eps, kernel="laplace" if kern == KERNEL_LAPLACE else "exp(-r)/r",
                         storage="valr" if eps >= 1e-6 else "f64",
                         stored_bytes=s["bytes_dense"] + s["bytes_factors"] + s["bytes_coupling"] + s["bytes_transfer"]))
        log(f"[bench] serve matrix {i}: {info[-1]} ({time.perf_counter() - t0:.0f}s)")
    S = hm.Server(mem_budget=args.serve_budget, max_slots=64, max_queue=100000, max_cols=64)
    ids = [S.register(M) for M in mats]
    Xpool = {}

    def block(m, r):
        key = (m, r)
        if key not in Xpool:
            Xpool[key] = gaussian_matrix(info[m]["n"], r, 7000 + 37 * m + r)
        return Xpool[key]

    def draw(k, seed):
        g = np.random.default_rng(seed)
        return [(int(g.integers(0, nm)), int(g.integers(1, 33))) for _ in range(k)]

    # capacity: a closed burst
    burst = draw(args.serve_requests, 4300)
    t1 = time.perf_counter()
    pend = [S.submit(ids[m], block(m, r))[0] for m, r in burst]
    for t in pend:
        S.wait(t)
    cap = len(burst) / (time.perf_counter() - t1)
    log(f"[bench] serve capacity {cap:.1f} requests/s")
    runs = []
    for frac in (0.5, 0.8, 1.0):
        reqs = draw(args.serve_requests, 4400 + int(frac * 10))
        gaps = np.random.default_rng(4200).exponential(1.0 / (frac * cap), size=len(reqs))
        pend, cols, bytes_ = [], 0, 0.0
        t1 = time.perf_counter()
        nxt = t1
        for (m, r), gap in zip(reqs, gaps):
            nxt += gap
            while time.perf_counter() < nxt:
                pass
            pend.append(S.submit(ids[m], block(m, r))[0])
            cols += r
            bytes_ += info[m]["stored_bytes"]
        lat = [S.wait(t)["latency_ms"] for t in pend]
        dt = time.perf_counter() - t1
        runs.append({"offered_fraction": frac, "offered_rps": round(frac * cap, 1), "requests": len(reqs),
                     "p50_ms": round(float(np.percentile(lat, 50)), 3),
                     "p99_ms": round(float(np.percentile(lat, 99)), 3),
                     "columns_per_s": round(cols / dt, 1), "requests_per_s": round(len(reqs) / dt, 1),
                     "GBs_if_unbatched": round(bytes_ / dt / 1e9, 1)})
        log(f"[bench] serve {runs[-1]}")
    st = S.stats()
    S.close()
    for M in mats:
        M.free()
    out = {"metric": "H-MVM serving p50/p99 latency + columns/s (hm_serve)", "value": runs[-1]["columns_per_s"],
           "unit": "columns/s", "n_gpus": 1, "steps": len(runs), "warmup": 0, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "mixed",
           "data": "synthetic (seeded sphere points, Laplace and exp(-r)/r kernels)",
           "config": {"workload": f"{nm} resident H/UH/H2 matrices, n ~ U[8192, {args.serve_nmax}], "
                                  "Poisson arrivals of 1..32-column requests", "matrices": info,
                      "mem_budget": args.serve_budget},
           "capacity_rps": round(cap, 1), "runs": runs, "server": st}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="h2_262144", choices=sorted(WORKLOADS))
    ap.add_argument("--legs", default=None, help="comma-separated storage legs (default per format)")
    ap.add_argument("--extra", default="uh32768,h2048",
                    help="comma-separated extra single-vector workloads reported beside the headline ('' = none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline leg")
    ap.add_argument("--no-parity", action="store_true", help="skip the oracle comparison of every leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, run a plain 1 GiB device copy (known traffic) to scale PMC counters")
    ap.add_argument("--copies-bytes", type=float, default=2.0e9,
                    help="upload copies until the rotated set exceeds this many bytes")
    ap.add_argument("--nrhs", default=None,
                    help="comma-separated block widths: run the many-right-hand-side path instead")
    ap.add_argument("--policies", default="f32,bf16", help="storage policies of the --nrhs runs")
    ap.add_argument("--no-tune", action="store_true", help="--nrhs runs: keep the default plan parameters")
    ap.add_argument("--serve", action="store_true", help="run the serving mix instead")
    ap.add_argument("--serve-matrices", type=int, default=16)
    ap.add_argument("--serve-nmax", type=int, default=131072, help="largest n of the serving mix")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-budget", type=float, default=4e9)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the product runs on one GPU only (--gpus {args.gpus} requested); "
              "sharding over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2405_03456_amd as hm
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)

    if args.serve:
        args.serve_budget = int(args.serve_budget)
        serve_mix(args, hm, torch)
        return
    if args.nrhs:
        fmt, n, eps, pseed, xseed, desc = WORKLOADS[args.workload]
        lay, st, vals, points = workload_inputs(hm, args.workload)
        many_rhs(args, hm, torch, lay, fmt, vals, eps, n, points, st, desc)
        return
    fmt = WORKLOADS[args.workload][0]
    legs = (args.legs or DEFAULT_LEGS[fmt]).split(",")
    if legs[0] != "f64":
        legs = ["f64"] + [leg for leg in legs if leg != "f64"]
    main_w = single_vector(args, hm, torch, args.workload, legs, not args.no_cpu, not args.no_parity)
    extras = {}
    for name in [w for w in args.extra.split(",") if w and w != args.workload]:
        extras[name] = single_vector(args, hm, torch, name, DEFAULT_LEGS[WORKLOADS[name][0]].split(","),
                                     False, not args.no_parity)

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] calibration: 3 copies of 1 GiB (read 1 GiB + write 1 GiB each)")

    f64 = main_w["legs"]["f64"]
    roof = f64["roofline"]
    if roof is not None:
        tr = measured_traffic(args.workload, "f64", roof["kernel"])
        roof["traffic"] = None if tr is None else int(tr)
    out = {
        "metric": METRIC,
        "value": f64["GBs"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded sphere points, Laplace kernel, ACA-compressed, nested bases)",
        "config": {"workload": main_w["workload"], "format": fmt, "n": main_w["n"], "eps": main_w["eps"],
                   "nrhs": 1, "storage": "f64", "accumulation": "f64", "rotated_copies": f64["copies"]},
        "matvecs_per_s": f64["matvecs_per_s"],
        "p10_ms": f64["p10_ms"],
        "p90_ms": f64["p90_ms"],
        "wall_ms_per_step": f64["wall_ms_per_step"],
        "timing": "graph replays, HIP events around each replay (median, p10, p90); roofline from "
                  "event-timed eager products with the dense stage running alone after the chain at its full "
                  "launch width (roofline.overlapped_avg_launch_us: the same kernel in the tuned, overlapped "
                  "schedule, legs[].dense_grid its workgroup cap)",
        "method_bytes_per_matvec": f64["method_bytes_per_matvec"],
        "overhead_bytes_per_matvec": f64["overhead_bytes_per_matvec"],
        "roofline": roof,
        "legs": main_w["legs"],
        "phases_f64": main_w["phases"]["f64"],
        # every leg's launches: [phase, tasks, average us]
        "phases_by_leg": {leg: [[p["name"], p["ntasks"], p["us_avg"]] for p in ph]
                          for leg, ph in main_w["phases"].items()},
    }
    if "cpu" in main_w:
        c = main_w["cpu"]
        out["cpu_baseline"] = {
            "value": round(c["all_cores"]["GBs"], 3), "unit": "GB/s", "cores": c["all_cores"]["threads"],
            "kind": "oracle", "matvecs_per_s": round(c["all_cores"]["matvecs_per_s"], 3),
            "one_core": {"GBs": round(c["one_core"]["GBs"], 3),
                         "matvecs_per_s": round(c["one_core"]["matvecs_per_s"], 3)},
            "host_triad_GBs": round(c["triad_GBs"], 1), "host_triad_threads": c["triad_threads"],
            "fraction_of_host_triad": round(c["all_cores"]["GBs"] / c["triad_GBs"], 3),
            "sample": f"median of 5 full FP64 {fmt.upper()} products of the same n={main_w['n']} matrix "
                      "(C/OpenMP oracle, oracle/mvm_omp.c), all cores and one core"}
    if extras:
        out["extra_workloads"] = {k: {"workload": v["workload"], "legs": v["legs"]} for k, v in extras.items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
