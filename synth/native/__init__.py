"""ctypes front end of the native input generator (lowrank.cpp)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "_synth_native.so")
_lib = None


def build(force: bool = False) -> str:
    src = os.path.join(HERE, "lowrank.cpp")
    if force or not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(src):
        subprocess.check_call(["g++", "-O3", "-march=x86-64-v2", "-fPIC", "-shared", "-std=c++17",
                               src, "-o", SO + ".tmp", "-lpthread"])
        os.replace(SO + ".tmp", SO)
    return SO


def _load():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(SO)
        vp, i64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        L.synth_dense_blocks.argtypes = [vp, i32, vp, i64, vp, i32]
        L.synth_dense_blocks.restype = None
        L.synth_lowrank.argtypes = [vp, i32, vp, i64, dbl, i32]
        L.synth_lowrank.restype = vp
        L.synth_lowrank_ranks.argtypes = [vp, vp]
        L.synth_lowrank_copy.argtypes = [vp, vp, vp, vp]
        L.synth_lowrank_free.argtypes = [vp]
        _lib = L
    return _lib


def _threads(n):
    return int(n) if n else min(16, os.cpu_count() or 1)


def dense_blocks(points, perm, kernel, coords, nthreads=0):
    L = _load()
    pc = np.ascontiguousarray(points[perm], dtype=np.float64)
    coords = np.ascontiguousarray(coords, dtype=np.int64).reshape(-1, 4)
    outs = [np.empty((int(c[1]), int(c[3])), order="F") for c in coords]
    ptrs = np.array([o.ctypes.data for o in outs], dtype=np.uint64)
    L.synth_dense_blocks(pc.ctypes.data, int(kernel), coords.ctypes.data, len(coords), ptrs.ctypes.data,
                         _threads(nthreads))
    return outs


def lowrank_blocks(points, perm, kernel, coords, eps, nthreads=0):
    """[(W, sigma, X)] per block, eps-truncated (ACA + recompression)."""
    L = _load()
    pc = np.ascontiguousarray(points[perm], dtype=np.float64)
    coords = np.ascontiguousarray(coords, dtype=np.int64).reshape(-1, 4)
    nb = len(coords)
    h = L.synth_lowrank(pc.ctypes.data, int(kernel), coords.ctypes.data, nb, float(eps), _threads(nthreads))
    try:
        ranks = np.zeros(nb, dtype=np.int32)
        L.synth_lowrank_ranks(h, ranks.ctypes.data)
        Ws = [np.empty((int(c[1]), int(k)), order="F") for c, k in zip(coords, ranks)]
        Ss = [np.empty(int(k)) for k in ranks]
        Xs = [np.empty((int(c[3]), int(k)), order="F") for c, k in zip(coords, ranks)]
        pw = np.array([a.ctypes.data for a in Ws], dtype=np.uint64)
        ps = np.array([a.ctypes.data for a in Ss], dtype=np.uint64)
        px = np.array([a.ctypes.data for a in Xs], dtype=np.uint64)
        L.synth_lowrank_copy(h, pw.ctypes.data, ps.ctypes.data, px.ctypes.data)
    finally:
        L.synth_lowrank_free(h)
    return list(zip(Ws, Ss, Xs))
