"""Oracle: the dense kernel matrix product (the matrix the H formats approximate).

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

Two implementations of the same definition, y[i] += alpha * sum_{j != i}
k(p_i, p_j) x[j] (Sec. 2.1; the diagonal of the point kernels is set to 0):
a numpy one that builds row panels explicitly, and a plain C loop
(dense_product.c, OpenMP over rows) for large n.  Vectors are in original
point order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle_dense.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile dense_product.c with gcc (-O2, OpenMP, no FMA contraction)."""
    src = os.path.join(_HERE, "dense_product.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               src, "-o", _SO + ".tmp", "-lm"])
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_dense_product.argtypes = [dp, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                             dp, dp, ip, ctypes.c_int64]
        lib.oracle_dense_product.restype = None
        lib.oracle_kernel_fro2.argtypes = [dp, ctypes.c_int64, ctypes.c_int]
        lib.oracle_kernel_fro2.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def kernel_rows(kernel: int, pts: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Explicit rows of the kernel matrix (original order), numpy."""
    P = np.asarray(pts, dtype=np.float64)
    R = P[rows]
    if kernel == 3:
        out = np.zeros((len(rows), len(P)))
        out[np.arange(len(rows)), rows] = 1.0
        return out
    if kernel == 2:
        out = np.ones((len(rows), len(P)))
    elif kernel == 4:
        out = (1.0 + R[:, 0])[:, None] * (2.0 + P[:, 1] * P[:, 2])[None, :]
    else:
        d = R[:, None, :] - P[None, :, :]
        r = np.sqrt((d * d).sum(axis=2))
        with np.errstate(divide="ignore", invalid="ignore"):
            out = 1.0 / (4.0 * np.pi * r) if kernel == 0 else np.exp(-r) / r
    out[np.arange(len(rows)), rows] = 0.0
    return out


def dense_product_numpy(kernel: int, pts: np.ndarray, alpha: float, x: np.ndarray,
                        y: np.ndarray, rows: np.ndarray | None = None, panel: int = 256) -> np.ndarray:
    n = len(pts)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.array(y, dtype=np.float64, copy=True)
    for i in range(0, len(rows), panel):
        r = rows[i:i + panel]
        out[r] += alpha * (kernel_rows(kernel, pts, r) @ x)
    return out


def dense_product(kernel: int, pts: np.ndarray, alpha: float, x: np.ndarray, y: np.ndarray,
                  rows: np.ndarray | None = None) -> np.ndarray:
    """y + alpha*A*x (restricted to `rows` if given; other entries copied)."""
    lib = _load()
    P = np.ascontiguousarray(pts, dtype=np.float64)
    n = len(P)
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    out = np.array(y, dtype=np.float64, copy=True)
    lib.oracle_dense_product(_ptr(P), n, int(kernel), float(alpha), _ptr(xx), _ptr(out),
                             _ptr(rows, ctypes.c_int64), len(rows))
    return out


def kernel_fro_norm(kernel: int, pts: np.ndarray) -> float:
    lib = _load()
    P = np.ascontiguousarray(pts, dtype=np.float64)
    return float(np.sqrt(lib.oracle_kernel_fro2(_ptr(P), len(P), int(kernel))))
