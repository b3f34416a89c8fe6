"""Oracle: the H / UH / H^2 products in plain C with OpenMP (mvm_omp.c).

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

The same product as oracle.mvm (eq. 4 over the stored blocks), evaluated
with the coefficient vectors of Sec. 3 (Alg. 4/6 forward transforms, eq. 5
coupling sums, the H^2 downward pass) and y written per leaf row cluster, so
that it runs in parallel on every host core.  It is the timed CPU baseline of
the benchmark and is checked against oracle.mvm by the tests.  Vectors at
this interface are in original point order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle_omp.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)


class _Tree(ctypes.Structure):
    _fields_ = [("nnodes", ctypes.c_int32), ("begin", _i64p), ("end", _i64p), ("level", _i32p),
                ("parent", _i32p), ("son0", _i32p), ("son1", _i32p), ("nblocks", ctypes.c_int64),
                ("tau", _i32p), ("sigma", _i32p), ("adm", _i32p)]


def build(force: bool = False) -> str:
    """Compile mvm_omp.c with gcc (-O2, OpenMP, no FMA contraction)."""
    src = os.path.join(_HERE, "mvm_omp.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               src, "-o", _SO + ".tmp"])
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        T = ctypes.POINTER(_Tree)
        vp = ctypes.c_void_p
        lib.oracle_h_mvm.argtypes = [T, vp, _i32p, vp, vp, vp, ctypes.c_double, _dp, _dp, ctypes.c_int]
        lib.oracle_uh_mvm.argtypes = [T, vp, _i32p, _i32p, vp, vp, vp, ctypes.c_double, _dp, _dp, ctypes.c_int]
        lib.oracle_h2_mvm.argtypes = [T, vp, _i32p, _i32p, vp, vp, vp, vp, vp, ctypes.c_double, _dp, _dp,
                                      ctypes.c_int]
        lib.oracle_triad.argtypes = [_dp, _dp, _dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int]
        for f in (lib.oracle_h_mvm, lib.oracle_uh_mvm, lib.oracle_h2_mvm, lib.oracle_triad):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class Prepared:
    """Tree arrays and per-block/per-node pointer tables of one stored
    matrix, kept alive between timed products."""

    def __init__(self, st, fmt: str, values):
        self.st, self.fmt = st, fmt
        keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a

        def ptrs(mats):
            addr = np.zeros(len(mats), dtype=np.uint64)
            for i, a in enumerate(mats):
                if a is None or np.size(a) == 0:
                    continue
                a = np.asfortranarray(a, dtype=np.float64)
                keep.append(a)
                addr[i] = a.ctypes.data
            keep.append(addr)
            return addr.ctypes.data

        def ranks(mats, axis):
            return arr([0 if a is None else (np.shape(a)[axis] if np.ndim(a) == 2 else len(a)) for a in mats],
                       np.int32)

        t = _Tree()
        t.nnodes = st.nnodes
        t.begin = arr(st.begin, np.int64).ctypes.data_as(_i64p)
        t.end = arr(st.end, np.int64).ctypes.data_as(_i64p)
        t.level = arr(st.level, np.int32).ctypes.data_as(_i32p)
        t.parent = arr(st.parent, np.int32).ctypes.data_as(_i32p)
        t.son0 = arr(st.son0, np.int32).ctypes.data_as(_i32p)
        t.son1 = arr(st.son1, np.int32).ctypes.data_as(_i32p)
        t.nblocks = st.nblocks
        t.tau = arr(st.blk_tau, np.int32).ctypes.data_as(_i32p)
        t.sigma = arr(st.blk_sigma, np.int32).ctypes.data_as(_i32p)
        t.adm = arr(st.blk_adm, np.int32).ctypes.data_as(_i32p)
        self.tree = t
        v = values
        self.dense = ptrs(v.dense)
        if fmt == "h":
            self.args = (arr(ranks(v.sigma, 0), np.int32).ctypes.data_as(_i32p), ptrs(v.W), ptrs(v.sigma),
                         ptrs(v.X))
        elif fmt == "uh":
            self.args = (ranks(v.row_basis, 1).ctypes.data_as(_i32p), ranks(v.col_basis, 1).ctypes.data_as(_i32p),
                         ptrs(v.row_basis), ptrs(v.col_basis), ptrs(v.coupling))
        else:
            self.args = (arr(v.row_rank, np.int32).ctypes.data_as(_i32p),
                         arr(v.col_rank, np.int32).ctypes.data_as(_i32p), ptrs(v.row_leaf_basis),
                         ptrs(v.row_transfer), ptrs(v.col_leaf_basis), ptrs(v.col_transfer), ptrs(v.coupling))
        self.keep = keep

    def product(self, alpha: float, x: np.ndarray, y: np.ndarray, threads: int = 0):
        """(y + alpha*M*x in original order, threads that ran); threads 0 =
        OpenMP's default (every core the process may use)."""
        lib = _load()
        perm = self.st.perm
        xc = np.ascontiguousarray(np.asarray(x, dtype=np.float64)[perm])
        yc = np.ascontiguousarray(np.asarray(y, dtype=np.float64)[perm])
        nt = int(threads) if threads else len(os.sched_getaffinity(0))
        f = {"h": lib.oracle_h_mvm, "uh": lib.oracle_uh_mvm, "h2": lib.oracle_h2_mvm}[self.fmt]
        used = f(ctypes.byref(self.tree), self.dense, *self.args, float(alpha), xc.ctypes.data_as(_dp),
                 yc.ctypes.data_as(_dp), nt)
        out = np.empty_like(yc)
        out[perm] = yc
        return out, used


def product(st, fmt: str, values, alpha: float, x: np.ndarray, y: np.ndarray, threads: int = 0) -> np.ndarray:
    return Prepared(st, fmt, values).product(alpha, x, y, threads)[0]


def triad_gbs(nbytes: float = 2.0e9, reps: int = 5, threads: int = 0):
    """Host bandwidth probe a = b + q c over three float64 arrays of
    nbytes/3 each: (median GB/s counting 24 bytes per element, threads)."""
    import time
    lib = _load()
    n = int(nbytes // 24)
    a, b, c = np.zeros(n), np.ones(n), np.full(n, 2.0)
    nt = int(threads) if threads else len(os.sched_getaffinity(0))
    lib.oracle_triad(a.ctypes.data_as(_dp), b.ctypes.data_as(_dp), c.ctypes.data_as(_dp), 3.0, n, nt)
    ts = []
    used = nt
    for _ in range(reps):
        t0 = time.perf_counter()
        used = lib.oracle_triad(a.ctypes.data_as(_dp), b.ctypes.data_as(_dp), c.ctypes.data_as(_dp), 3.0, n, nt)
        ts.append(time.perf_counter() - t0)
    return 24.0 * n / float(np.median(ts)) / 1e9, used
