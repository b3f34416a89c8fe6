"""MI355X (gfx950) engine for the hierarchical-matrix product y += alpha*M*x.

Thin Python binding over the C ABI of libhm.so (include/hm.h): argument
marshalling only, every step of the product runs in the library's HIP
kernels.  PyTorch is used for device memory and streams.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (HM_ACC_AUTO, HM_ACC_F32, HM_ACC_F64, HM_BF16, HM_CLUSTER_ORDER,  # noqa: F401
                   HM_F16, HM_F32, HM_F64, HM_FMT_H, HM_FMT_H2, HM_FMT_UH, HM_FP8E4M3, HM_VALR_AUTO,
                   HMError)

FORMATS = {"h": HM_FMT_H, "uh": HM_FMT_UH, "h2": HM_FMT_H2}
PARTITIONS = {"standard": _lib.HM_PART_STANDARD, "hodlr": _lib.HM_PART_HODLR, "blr": _lib.HM_PART_BLR}
DTYPES = {"f64": HM_F64, "f32": HM_F32, "bf16": HM_BF16, "f16": HM_F16, "fp8": HM_FP8E4M3,
          "valr": HM_VALR_AUTO,
          # byte-aligned codecs (Sec. 4.1): fixed formats and the adaptive policies
          "fpx24": _lib.HM_FPX24, "fpx40": _lib.HM_FPX40, "fpx48": _lib.HM_FPX48, "fpx56": _lib.HM_FPX56,
          "aflp8": _lib.HM_AFLP8, "aflp16": _lib.HM_AFLP16, "aflp24": _lib.HM_AFLP24,
          "aflp32": _lib.HM_AFLP32, "aflp40": _lib.HM_AFLP40, "aflp48": _lib.HM_AFLP48,
          "aflp56": _lib.HM_AFLP56, "aflp": _lib.HM_AFLP_AUTO, "fpx": _lib.HM_FPX_AUTO}
DTYPE_NAMES = {v: k for k, v in DTYPES.items()}


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Layout:
    """Cluster tree + block tree built by the library (hm_build_layout)."""

    def __init__(self, points, leaf_size: int = 64, eta: float = 2.0, partition: str = "standard"):
        L = _lib.lib()
        self._pts = np.ascontiguousarray(points, dtype=np.float64)
        if self._pts.ndim != 2 or self._pts.shape[1] != 3:
            raise ValueError("points must be n x 3")
        opts = _lib.LayoutOpts(leaf_size, eta, PARTITIONS[partition])
        h = ctypes.c_void_p()
        _lib.check(L.hm_build_layout(_dptr(self._pts), self._pts.shape[0], ctypes.byref(opts),
                                     ctypes.byref(h)))
        self._h = h
        self.n = self._pts.shape[0]

    @property
    def handle(self):
        return self._h

    def export(self) -> dict:
        """Copies of the layout arrays (see hm_layout_view)."""
        v = _lib.LayoutView()
        _lib.check(_lib.lib().hm_layout_export(self._h, ctypes.byref(v)))

        def arr(p, count, dt):
            return np.ctypeslib.as_array(p, shape=(count,)).astype(dt, copy=True) if count else np.zeros(0, dt)
        N, B = v.nnodes, v.nblocks
        return dict(n=v.n, depth=v.depth, perm=arr(v.perm, v.n, np.int64),
                    begin=arr(v.node_begin, N, np.int64), end=arr(v.node_end, N, np.int64),
                    level=arr(v.node_level, N, np.int64), parent=arr(v.node_parent, N, np.int64),
                    son0=arr(v.node_son0, N, np.int64), son1=arr(v.node_son1, N, np.int64),
                    blk_tau=arr(v.blk_tau, B, np.int64), blk_sigma=arr(v.blk_sigma, B, np.int64),
                    blk_adm=arr(v.blk_adm, B, np.int64).astype(bool))

    def stats(self) -> dict:
        """Partition statistics per level (hm_layout_stats); no values needed."""
        s = _lib.LayoutInfo()
        _lib.check(_lib.lib().hm_layout_stats(self._h, ctypes.byref(s)))
        out = {}
        for k, _ in _lib.LayoutInfo._fields_:
            v = getattr(s, k)
            out[k] = list(v)[: s.depth + 1] if k.endswith("_per_level") else v
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None and _lib._lib is not None:
            _lib._lib.hm_layout_free(h)
            self._h = None


class _PtrTable:
    """Array of double* (one per node/block) keeping the arrays alive."""

    def __init__(self, arrays):
        self.keep = []
        self.addr = np.zeros(len(arrays), dtype=np.uint64)
        for i, a in enumerate(arrays):
            if a is None:
                continue
            a = np.asfortranarray(a, dtype=np.float64)
            if a.size == 0:
                continue
            self.keep.append(a)
            self.addr[i] = a.ctypes.data

    @property
    def ptr(self):
        return self.addr.ctypes.data


def _ranks(arrays, axis=1):
    return np.array([0 if a is None else (a.shape[axis] if np.ndim(a) == 2 else len(a)) for a in arrays],
                    dtype=np.int32)


def marshal_values(fmt: str, values):
    """hm_values for `values` (see Matrix) plus the arrays that must stay alive."""
    f = FORMATS[fmt]
    v = _lib.Values()
    tabs = []

    def tab(arrs):
        t = _PtrTable(arrs)
        tabs.append(t)
        return t.ptr

    def ints(a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        tabs.append(a)
        return a.ctypes.data

    v.dense = tab(values.dense)
    if f == HM_FMT_H:
        v.rank = ints(_ranks(values.sigma, 0))
        v.W, v.sigma, v.X = tab(values.W), tab(values.sigma), tab(values.X)
    elif f == HM_FMT_UH:
        v.row_rank = ints(_ranks(values.row_basis))
        v.col_rank = ints(_ranks(values.col_basis))
        v.row_basis, v.col_basis = tab(values.row_basis), tab(values.col_basis)
        v.coupling = tab(values.coupling)
    else:
        v.row_rank, v.col_rank = ints(values.row_rank), ints(values.col_rank)
        v.row_basis, v.col_basis = tab(values.row_leaf_basis), tab(values.col_leaf_basis)
        v.row_transfer, v.col_transfer = tab(values.row_transfer), tab(values.col_transfer)
        v.coupling = tab(values.coupling)
    if f != HM_FMT_H:
        # basis weights for VALR (optional)
        if getattr(values, "row_sv", None) is not None:
            v.row_sv = tab(values.row_sv)
        if getattr(values, "col_sv", None) is not None:
            v.col_sv = tab(values.col_sv)
    return v, tabs


def make_precision(eps=0.0, dense="f64", diag=None, factor="f64", coupling=None, accum=HM_ACC_AUTO):
    return _lib.Precision(eps, DTYPES[dense], DTYPES[diag or dense], DTYPES[factor],
                          DTYPES[coupling or factor], accum)


SCHEDULES = {"persistent": _lib.HM_SCHED_PERSISTENT, "staged": _lib.HM_SCHED_STAGED}
H2_LEVELS = {"coupling_first": 0, "per_level": 1}
SYNCS = {"owner": 0, "atomic": 1, "private": 2}


def make_opts(task_bytes: int = 0, spread_dense: bool = False, dense_grid: int = 0, fork_after: int = 0,
              valr_promote: bool = False, schedule: str = "staged", dense_after: int = 0,
              spin_limit_us: int = 0, tickets_per_grab: int = 0, adjoint: bool = False, sync: str = "owner",
              h2_levels: str = "coupling_first", chain_task_bytes: int = 0):
    """hm_upload_opts (all zero = the library's defaults).  h2_levels:
    "coupling_first" (every level's couplings in one launch after the up
    pass) or "per_level" (couplings with the transfers of their level)."""
    return _lib.UploadOpts(int(task_bytes), int(bool(spread_dense)), int(dense_grid), int(fork_after),
                           int(bool(valr_promote)), SCHEDULES[schedule], int(dense_after), int(spin_limit_us),
                           int(tickets_per_grab), SYNCS[sync], int(bool(adjoint)), H2_LEVELS[h2_levels],
                           int(chain_task_bytes))


def _stats_dict(s) -> dict:
    out = {k: getattr(s, k) for k, _ in _lib.Stats._fields_}
    out["bytes_per_dtype"] = list(s.bytes_per_dtype)
    out["entries_per_dtype"] = list(s.entries_per_dtype)
    return out


def plan_stats(layout: "Layout", fmt: str, values, eps: float = 0.0, dense="f64", diag=None,
               factor="f64", coupling=None, accum: int = HM_ACC_AUTO, **opts) -> dict:
    """Storage statistics hm_upload would produce, computed on the host
    only (hm_plan_stats): no device memory is touched.  `opts` are the
    hm_upload_opts fields (see make_opts)."""
    v, tabs = marshal_values(fmt, values)
    prec = make_precision(eps, dense, diag, factor, coupling, accum)
    o = make_opts(**opts)
    s = _lib.Stats()
    _lib.check(_lib.lib().hm_plan_stats(layout.handle, FORMATS[fmt], ctypes.byref(v), ctypes.byref(prec),
                                        ctypes.byref(o), ctypes.byref(s)))
    del tabs
    return _stats_dict(s)


class Matrix:
    """A hierarchical matrix uploaded to the current HIP device (hm_upload).

    `values` is any object with the attributes of the chosen format:
      h:  dense, W, sigma, X                       (per block)
      uh: dense, row_basis, col_basis, coupling    (per block / node)
      h2: dense, row_rank, col_rank, row_leaf_basis, row_transfer,
          col_leaf_basis, col_transfer, coupling
    and for VALR storage ("valr") of UH/H2 bases also row_sv, col_sv.
    Keyword `opts` are the engine options of hm_upload_opts (make_opts).
    """

    def __init__(self, layout: Layout, fmt: str, values, eps: float = 0.0, dense="f64", diag=None,
                 factor="f64", coupling=None, accum: int = HM_ACC_AUTO, stream=None, **opts):
        L = _lib.lib()
        self.layout = layout
        self.fmt = fmt
        f = FORMATS[fmt]
        v, tabs = marshal_values(fmt, values)
        prec = make_precision(eps, dense, diag, factor, coupling, accum)
        o = make_opts(**opts)
        h = ctypes.c_void_p()
        _lib.check(L.hm_upload(layout.handle, f, ctypes.byref(v), ctypes.byref(prec), ctypes.byref(o),
                               _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = _lib.Stats()
        _lib.check(_lib.lib().hm_matrix_stats(self._h, ctypes.byref(s)))
        return _stats_dict(s)

    def mvm(self, x, y, alpha: float = 1.0, cluster_order: bool = False, stream=None, timing: bool = False,
            adjoint: bool = False):
        """y += alpha * M * x (or M^T x with adjoint=True) for device float64
        tensors (enqueued, asynchronous)."""
        xp, yp = _dev_ptr(x, self.layout.n), _dev_ptr(y, self.layout.n)
        flags = (HM_CLUSTER_ORDER if cluster_order else 0) | (_lib.HM_TIMING if timing else 0) | \
            (_lib.HM_ADJOINT if adjoint else 0)
        _lib.check(_lib.lib().hm_mvm(self._h, float(alpha), xp, yp, flags, _stream_ptr(stream)))

    def mvm_many(self, X, Y, alpha: float = 1.0, cluster_order: bool = False, stream=None, timing: bool = False):
        """Y += alpha * M * X for an n x r block (column-major device tensors)."""
        mvm_batch([self], [X], [Y], alpha, cluster_order, stream, timing)

    def tune(self, nrhs: int, vec_dtype: str = "f64", reps: int = 3, stream=None) -> dict:
        """Pick the many-RHS plan parameters for blocks of `nrhs` columns (hm_tune_batch)."""
        r = _lib.TuneResult()
        _lib.check(_lib.lib().hm_tune_batch(self._h, int(nrhs), DTYPES[vec_dtype], int(reps),
                                            _stream_ptr(stream), ctypes.byref(r)))
        return dict(target_bytes=r.target_bytes, nrb=r.nrb, ms=r.ms, ncandidates=r.ncandidates)

    def tune_mvm(self, reps: int = 10, stream=None) -> dict:
        """Pick the single-vector schedule and its parameter (hm_tune_mvm)."""
        r = _lib.TuneMvmResult()
        _lib.check(_lib.lib().hm_tune_mvm(self._h, int(reps), _stream_ptr(stream), ctypes.byref(r)))
        return dict(fork_after=r.fork_after, ncandidates=r.ncandidates, ms=r.ms, ms_first=r.ms_first,
                    schedule="persistent" if r.schedule == _lib.HM_SCHED_PERSISTENT else "staged",
                    dense_after=r.dense_after, ms_staged=r.ms_staged, ms_persistent=r.ms_persistent,
                    fork2=r.fork2, dense_split=r.dense_split, dense_grid=r.dense_grid)

    def set_schedule(self, schedule: str, param: int = 0):
        """hm_set_schedule: "staged" (param = fork point) or "persistent"
        (param = dense_after)."""
        _lib.check(_lib.lib().hm_set_schedule(self._h, SCHEDULES[schedule], int(param)))

    def set_dense_split(self, fork2: int, first_tasks: int):
        """hm_set_dense_split: the dense stage as two launches (first_tasks
        tasks from the fork point, the rest after fork2 dependent stages);
        first_tasks = 0 restores one launch."""
        _lib.check(_lib.lib().hm_set_dense_split(self._h, int(fork2), int(first_tasks)))

    def check(self):
        """Wait for the device; raise if a persistent launch of this matrix
        was aborted since the last check (hm_matrix_check)."""
        _lib.check(_lib.lib().hm_matrix_check(self._h))

    def graph(self, x, y, alpha: float = 1.0, cluster_order: bool = False, stream=None,
              adjoint: bool = False) -> "Graph":
        """Capture one product (fixed x, y, alpha) into a replayable HIP graph."""
        return Graph(self, x, y, alpha, cluster_order, stream, adjoint)

    def timing(self) -> list:
        """Per-phase kernel times of the calls made with timing=True (and clears them)."""
        cap = 4096
        arr = (_lib.PhaseTiming * cap)()
        n = ctypes.c_int32()
        _lib.check(_lib.lib().hm_timing_read(self._h, arr, cap, ctypes.byref(n)))
        return [dict(name=arr[i].name.decode(), ms_total=arr[i].ms_total, launches=arr[i].launches,
                     algorithmic_bytes=arr[i].algorithmic_bytes, ntasks=arr[i].ntasks, nowners=arr[i].nowners,
                     data_bytes=arr[i].data_bytes, data_entries=arr[i].data_entries, nrhs=arr[i].nrhs,
                     method_bytes=arr[i].method_bytes)
                for i in range(min(n.value, cap))]

    def free(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None and _lib._lib is not None:
            _lib._lib.hm_matrix_free(h)
        self._h = None

    def __del__(self):
        self.free()


def _block_arg(t, n, name):
    """(device pointer, leading dimension, columns, vec dtype) of a vector
    block: a 1-D tensor of length n, or an n x r column-major tensor."""
    import torch
    if not t.is_cuda or t.dtype not in (torch.float64, torch.float32):
        raise ValueError(f"{name} must be a float64 or float32 device tensor")
    vdt = HM_F64 if t.dtype == torch.float64 else HM_F32
    if t.dim() == 1:
        if t.numel() != n or t.stride(0) != 1:
            raise ValueError(f"{name}: contiguous vector of length n expected")
        return t.data_ptr(), n, 1, vdt
    if t.dim() != 2 or t.shape[0] != n or (t.shape[1] > 1 and t.stride(0) != 1):
        raise ValueError(f"{name} must be n x r and column-major (e.g. x.T.contiguous().T)")
    ld = t.stride(1) if t.shape[1] > 1 else n
    return t.data_ptr(), max(ld, n), t.shape[1], vdt


def _marshal_batch(mats, X, Y):
    k = len(mats)
    if len(X) != k or len(Y) != k:
        raise ValueError("mats, X and Y must have the same length")
    hs = (ctypes.c_void_p * k)()
    xs, ys = (ctypes.c_void_p * k)(), (ctypes.c_void_p * k)()
    ldx, ldy = (ctypes.c_int64 * k)(), (ctypes.c_int64 * k)()
    nr = (ctypes.c_int32 * k)()
    vdt = None
    for i, (M, x, y) in enumerate(zip(mats, X, Y)):
        px, lx, rx, dx = _block_arg(x, M.layout.n, "X")
        py, ly, ry, dy = _block_arg(y, M.layout.n, "Y")
        if rx != ry or dx != dy or (vdt is not None and dx != vdt):
            raise ValueError("X and Y blocks must agree in width and all share one dtype")
        vdt = dx
        hs[i], xs[i], ys[i], ldx[i], ldy[i], nr[i] = M.handle.value, px, py, lx, ly, rx
    return k, hs, xs, ldx, nr, ys, ldy, HM_F64 if vdt is None else vdt


def mvm_batch(mats, X, Y, alpha: float = 1.0, cluster_order: bool = False, stream=None, timing: bool = False,
              adjoint: bool = False):
    """Y[i] += alpha * mats[i] * X[i] for every i (hm_mvm_batch; mats[i]^T
    with adjoint=True).  X[i], Y[i]: device tensors of n_i x r_i values
    (column-major) or vectors of length n_i, all float64 or all float32."""
    k, hs, xs, ldx, nr, ys, ldy, vdt = _marshal_batch(mats, X, Y)
    flags = (HM_CLUSTER_ORDER if cluster_order else 0) | (_lib.HM_TIMING if timing else 0) | \
        (_lib.HM_ADJOINT if adjoint else 0)
    _lib.check(_lib.lib().hm_mvm_batch(hs, k, float(alpha), xs, ldx, nr, ys, ldy, vdt, flags,
                                       _stream_ptr(stream)))


def mvm_batch_noalloc(mats, X, Y, alpha: float = 1.0, cluster_order: bool = False, stream=None):
    """hm_mvm_batch_noalloc: the products of mvm_batch with the workspaces
    taken from the library's fixed device array (nothing is allocated)."""
    k, hs, xs, ldx, nr, ys, ldy, vdt = _marshal_batch(mats, X, Y)
    flags = HM_CLUSTER_ORDER if cluster_order else 0
    _lib.check(_lib.lib().hm_mvm_batch_noalloc(hs, k, float(alpha), xs, ldx, nr, ys, ldy, vdt, flags,
                                               _stream_ptr(stream)))


class BatchGraph:
    """hm_graph_create_batch: one captured hm_mvm_batch call, replayed with launch()."""

    def __init__(self, mats, X, Y, alpha: float = 1.0, cluster_order: bool = False, stream=None,
                 adjoint: bool = False):
        self._keep = (list(mats), list(X), list(Y))
        k, hs, xs, ldx, nr, ys, ldy, vdt = _marshal_batch(mats, X, Y)
        h = ctypes.c_void_p()
        flags = (HM_CLUSTER_ORDER if cluster_order else 0) | (_lib.HM_ADJOINT if adjoint else 0)
        _lib.check(_lib.lib().hm_graph_create_batch(hs, k, float(alpha), xs, ldx, nr, ys, ldy, vdt, flags,
                                                    _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _lib.check(_lib.lib().hm_graph_launch(self._h, _stream_ptr(stream)))

    def free(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None and _lib._lib is not None:
            _lib._lib.hm_graph_free(h)
        self._h = None

    def __del__(self):
        self.free()


class Graph:
    """hm_graph: a captured product, replayed with launch()."""

    def __init__(self, M: Matrix, x, y, alpha, cluster_order, stream, adjoint=False):
        self.matrix = M           # keeps the matrix alive
        self._xy = (x, y)         # keeps the vectors alive
        h = ctypes.c_void_p()
        flags = (HM_CLUSTER_ORDER if cluster_order else 0) | (_lib.HM_ADJOINT if adjoint else 0)
        _lib.check(_lib.lib().hm_graph_create(M.handle, float(alpha), _dev_ptr(x, M.layout.n),
                                              _dev_ptr(y, M.layout.n), flags, _stream_ptr(stream),
                                              ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _lib.check(_lib.lib().hm_graph_launch(self._h, _stream_ptr(stream)))

    def free(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None and _lib._lib is not None:
            _lib._lib.hm_graph_free(h)
        self._h = None

    def __del__(self):
        self.free()


class Server:
    """hm_serve_*: a request loop over resident matrices (continuous batching)."""

    def __init__(self, mem_budget: int = 1 << 30, max_slots: int = 64, max_queue: int = 4096, max_cols: int = 64,
                 fake: bool = False, fake_us: int = 0):
        opts = _lib.ServeOpts(int(mem_budget), int(max_slots), int(max_queue), int(max_cols), 1 if fake else 0,
                              int(fake_us))
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().hm_serve_create(ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._pending = {}    # ticket -> (X, Y) kept alive until done
        self._mats = []

    def register(self, M: "Matrix") -> int:
        i = ctypes.c_int32()
        _lib.check(_lib.lib().hm_serve_register(self._h, M.handle, ctypes.byref(i)))
        self._mats.append(M)
        return i.value

    def register_shape(self, n: int) -> int:
        i = ctypes.c_int32()
        _lib.check(_lib.lib().hm_serve_register_shape(self._h, int(n), ctypes.byref(i)))
        return i.value

    def submit(self, mid: int, X, alpha: float = 1.0):
        """Queue Y := alpha * M * X for a host n x r (or length-n) float64 block;
        returns (ticket, Y) where Y is filled once poll() reports done."""
        X = np.asfortranarray(X, dtype=np.float64)
        r = 1 if X.ndim == 1 else X.shape[1]
        Y = np.zeros(X.shape, dtype=np.float64, order="F")
        t = ctypes.c_uint64()
        _lib.check(_lib.lib().hm_serve_submit(self._h, int(mid), float(alpha), X.ctypes.data, r, Y.ctypes.data,
                                              ctypes.byref(t)))
        self._pending[t.value] = (X, Y)
        return t.value, Y

    def poll(self, ticket: int):
        """None while queued/running, else the request's stats (dict)."""
        done = ctypes.c_int32()
        st = _lib.ReqStats()
        status = _lib.lib().hm_serve_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(st))
        if status != _lib.HM_OK:
            self._pending.pop(ticket, None)
            _lib.check(status)
        if not done.value:
            return None
        self._pending.pop(ticket, None)
        return {k: getattr(st, k) for k, _ in _lib.ReqStats._fields_}

    def wait(self, ticket: int, timeout_s: float = 120.0):
        import time
        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"ticket {ticket} not done after {timeout_s} s")
            time.sleep(20e-6)

    def stats(self) -> dict:
        s = _lib.ServeStats()
        _lib.check(_lib.lib().hm_serve_stats_read(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in _lib.ServeStats._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None and _lib._lib is not None:
            _lib._lib.hm_serve_destroy(h)
        self._h = None
        self._pending = {}

    def __del__(self):
        self.close()


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t, n):
    if isinstance(t, int):
        return t
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n):
        raise ValueError("vectors must be contiguous float64 device tensors of length n")
    return t.data_ptr()


def round_host(dtype: str, values) -> np.ndarray:
    """The library's storage rounding (host), for tests."""
    a = np.ascontiguousarray(values, dtype=np.float64)
    out = np.empty_like(a)
    _lib.check(_lib.lib().hm_round_host(DTYPES[dtype], _dptr(a), _dptr(out), a.size))
    return out


def codec_column(dtype: str, values, eps: float = 0.0, ebits: int = 0):
    """The library's storage of one column (host, for tests): (stored values,
    code words, {"dtype", "bytes", "ebits", "k"})."""
    a = np.ascontiguousarray(values, dtype=np.float64)
    out = np.empty_like(a)
    codes = np.zeros(a.size, dtype=np.uint64)
    info = (ctypes.c_int32 * 4)()
    _lib.check(_lib.lib().hm_codec_column(DTYPES[dtype], float(eps), int(ebits), _dptr(a), a.size, _dptr(out),
                                          codes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), info))
    return out, codes, {"dtype": DTYPE_NAMES[info[0]], "bytes": info[1], "ebits": info[2], "k": info[3]}


def version() -> str:
    return _lib.lib().hm_version().decode()
