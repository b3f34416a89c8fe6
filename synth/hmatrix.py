"""Compression of a kernel matrix into H, uniform-H and H^2 form.

This module produces the *stored matrix*, the input of the product.  The
paper takes the H-matrix as given and only cites construction methods
(Sec. 2.2-2.4), so the steps below are one reasonable choice, written once and
consumed identically by the oracle and the GPU path (both receive the same
factors, keyed by block).

* H (Sec. 2.2, eq. 3): every admissible block M_b gets a truncated SVD
  W_b diag(s_b) X_b^T with the Frobenius rule
  sqrt(sum_{i>=k} s_i^2) <= eps * ||M_b||_F.  Small problems use LAPACK's
  exact SVD; large ones use adaptive cross approximation followed by a
  QR/SVD recompression (native code, same truncation rule).
* UH (Sec. 2.3): the row basis of tau is the eps-truncated left singular
  space of the stack [W_b diag(s_b)/||s_b||] over the low-rank blocks in the
  block row of tau; column bases alike with X_b; couplings
  S_b = (Wt_tau^T W_b) diag(s_b) (X_b^T Xt_sigma).
* H^2 (Sec. 2.4): nested bases built as "total cluster bases": a top-down
  condensation of every block row restricted to tau (including the
  ancestors' rows), then a bottom-up pass that takes leaf bases from the
  condensed data and inner bases as blkdiag(W_t0, W_t1) Q with Q from an SVD
  of the sons' projected data; the transfer matrices are the two row slices
  of Q.  Ranks vary per cluster, so E_t' is k_t' x k_t.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .inputs import Structure, kernel_block


def _trunc_rank(sv: np.ndarray, tol_abs: float) -> int:
    """Smallest k with sqrt(sum_{i>=k} sv_i^2) <= tol_abs."""
    if len(sv) == 0:
        return 0
    # tail[k] = sqrt(sum_{i>=k} sv_i^2), computed from the end
    tail2 = np.cumsum((sv * sv)[::-1])[::-1]
    tail2 = np.append(tail2, 0.0)
    ok = np.nonzero(tail2 <= tol_abs * tol_abs)[0]
    return int(ok[0])


@dataclass
class HValues:
    kernel: int
    eps: float
    dense: list          # per block: F-order array (nrows x ncols) or None
    W: list              # per block: nrows x k (orthonormal columns) or None
    sigma: list          # per block: k singular values or None
    X: list              # per block: ncols x k (orthonormal columns) or None

    def rank(self, b: int) -> int:
        return 0 if self.sigma[b] is None else len(self.sigma[b])


@dataclass
class UHValues:
    kernel: int
    eps: float
    dense: list          # per block
    row_basis: list      # per node: |tau| x k_tau
    row_sv: list         # per node: k_tau weights (singular values of the stack)
    col_basis: list
    col_sv: list
    coupling: list       # per block: k_tau x k_sigma for admissible blocks


@dataclass
class H2Values:
    kernel: int
    eps: float
    dense: list
    row_rank: np.ndarray
    col_rank: np.ndarray
    row_leaf_basis: list   # per node: |tau| x k_tau at leaves, None elsewhere
    row_transfer: list     # per node: k_tau x k_parent (None at the root)
    col_leaf_basis: list
    col_transfer: list
    row_sv: list
    col_sv: list
    coupling: list


def _points_cluster_order(points: np.ndarray, st: Structure) -> np.ndarray:
    return np.ascontiguousarray(points[st.perm])


def dense_block(points_c: np.ndarray, kernel: int, st: Structure, b: int) -> np.ndarray:
    t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
    r0, r1, c0, c1 = st.begin[t], st.end[t], st.begin[s], st.end[s]
    rows = np.arange(r0, r1)
    cols = np.arange(c0, c1)
    return kernel_block(kernel, points_c[r0:r1], points_c[c0:c1], rows, cols)


def compress_h(points: np.ndarray, kernel: int, st: Structure, eps: float,
               method: str = "auto", nthreads: int = 0) -> HValues:
    """Dense inadmissible leaves + eps-truncated low-rank admissible leaves."""
    if method == "auto":
        method = "svd" if st.n <= 8192 else "aca"
    pc = _points_cluster_order(points, st)
    nb = st.nblocks
    dense = [None] * nb
    W = [None] * nb
    sig = [None] * nb
    X = [None] * nb
    adm_ids = np.nonzero(st.blk_adm)[0]
    den_ids = np.nonzero(~st.blk_adm.astype(bool))[0]
    if method == "svd":
        for b in den_ids:
            dense[b] = dense_block(pc, kernel, st, int(b))
        for b in adm_ids:
            M = dense_block(pc, kernel, st, int(b))
            U, s, Vt = np.linalg.svd(M, full_matrices=False)
            fro = float(np.sqrt((s * s).sum()))
            k = _trunc_rank(s, eps * fro)
            W[b] = np.asfortranarray(U[:, :k])
            sig[b] = s[:k].copy()
            X[b] = np.asfortranarray(Vt[:k].T)
    elif method == "aca":
        from . import native
        coords = st.block_coords()
        dense_list = native.dense_blocks(points, st.perm, kernel, coords[den_ids], nthreads)
        for i, b in enumerate(den_ids):
            dense[b] = dense_list[i]
        lr = native.lowrank_blocks(points, st.perm, kernel, coords[adm_ids], eps, nthreads)
        for i, b in enumerate(adm_ids):
            W[b], sig[b], X[b] = lr[i]
    else:
        raise ValueError(method)
    return HValues(kernel, eps, dense, W, sig, X)


def _svd_left(Z: np.ndarray):
    if Z.shape[1] == 0 or Z.shape[0] == 0:
        return np.zeros((Z.shape[0], 0)), np.zeros(0)
    U, s, _ = np.linalg.svd(Z, full_matrices=False)
    return U, s


def to_uh(h: HValues, st: Structure, eps: float | None = None) -> UHValues:
    """Shared row/column cluster bases and coupling matrices."""
    eps = h.eps if eps is None else eps
    N = st.nnodes
    row_basis, row_sv, col_basis, col_sv = [None] * N, [None] * N, [None] * N, [None] * N
    rows_lr = st.row_blocks(True)
    cols_lr = st.col_blocks(True)
    for side, groups, fac, basis, svs in (("row", rows_lr, h.W, row_basis, row_sv),
                                          ("col", cols_lr, h.X, col_basis, col_sv)):
        def one(v, groups=groups, fac=fac, basis=basis, svs=svs):
            parts = []
            for b in groups.get(v, []):
                s = h.sigma[b]
                nrm = float(np.sqrt((s * s).sum())) if s is not None and len(s) else 0.0
                if nrm > 0.0:
                    parts.append(fac[b] * (s / nrm)[None, :])
            if parts:
                U, sv = _svd_left(np.hstack(parts))
                k = _trunc_rank(sv, eps)
                basis[v] = np.asfortranarray(U[:, :k])
                svs[v] = sv[:k].copy()
            else:
                basis[v] = np.zeros((st.size(v), 0), order="F")
                svs[v] = np.zeros(0)
        _levels(st, one, root_first=True)     # every node is independent
    coupling = [None] * st.nblocks
    for b in np.nonzero(st.blk_adm)[0]:
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        if h.sigma[b] is None or len(h.sigma[b]) == 0:
            coupling[b] = np.zeros((row_basis[t].shape[1], col_basis[s].shape[1]), order="F")
            continue
        L = row_basis[t].T @ h.W[b]
        R = h.X[b].T @ col_basis[s]
        coupling[b] = np.asfortranarray((L * h.sigma[b][None, :]) @ R)
    return UHValues(h.kernel, eps, list(h.dense), row_basis, row_sv, col_basis, col_sv, coupling)


def _levels(st: Structure, fn, root_first: bool) -> None:
    """fn(v) for every node, one tree level after the other (root first or
    leaves first); the nodes of one level are independent and run on a
    thread pool (LAPACK releases the GIL), with one BLAS thread each."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    lv = np.asarray(st.level)
    levels = range(int(lv.max()) + 1) if root_first else range(int(lv.max()), -1, -1)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with threadpool_limits(limits=1), ThreadPoolExecutor(max_workers=workers) as ex:
        for lev in levels:
            nodes = [int(v) for v in np.nonzero(lv == lev)[0]]
            list(ex.map(fn, nodes))


def _nested_side(st: Structure, groups: dict, fac: list, sigma: list, eps: float, cond_eps: float):
    """Nested basis for one side.  Returns explicit bases per node (for the
    couplings), ranks, leaf bases, transfers and leaf singular values."""
    N = st.nnodes
    cond = [None] * N

    def condense(v):
        parts = []
        for b in groups.get(v, []):
            s = sigma[b]
            nrm = float(np.sqrt((s * s).sum())) if s is not None and len(s) else 0.0
            if nrm > 0.0:
                parts.append(fac[b] * (s / nrm)[None, :])
        p = int(st.parent[v])
        if p >= 0 and cond[p] is not None and cond[p].shape[1] > 0:
            off = int(st.begin[v] - st.begin[p])
            parts.append(cond[p][off:off + st.size(v)])
        if parts:
            U, sv = _svd_left(np.hstack(parts))
            r = _trunc_rank(sv, cond_eps)
            cond[v] = U[:, :r] * sv[:r][None, :]
        else:
            cond[v] = np.zeros((st.size(v), 0))

    explicit = [None] * N
    rank = np.zeros(N, dtype=np.int64)
    leaf_basis = [None] * N
    transfer = [None] * N
    svals = [None] * N

    def nest(v):
        if st.is_leaf(v):
            U, sv = _svd_left(cond[v])
            k = _trunc_rank(sv, eps)
            explicit[v] = np.asfortranarray(U[:, :k])
            leaf_basis[v] = explicit[v]
            svals[v] = sv[:k].copy()
            rank[v] = k
        else:
            s0, s1 = st.sons(v)
            n0 = st.size(s0)
            C = cond[v]
            top = explicit[s0].T @ C[:n0]
            bot = explicit[s1].T @ C[n0:]
            Chat = np.vstack([top, bot])
            U, sv = _svd_left(Chat)
            k = _trunc_rank(sv, eps)
            Q = U[:, :k]
            k0 = explicit[s0].shape[1]
            transfer[s0] = np.asfortranarray(Q[:k0])
            transfer[s1] = np.asfortranarray(Q[k0:])
            explicit[v] = np.asfortranarray(np.vstack([explicit[s0] @ transfer[s0],
                                                       explicit[s1] @ transfer[s1]]))
            svals[v] = sv[:k].copy()
            rank[v] = k
        cond[v] = None if not st.is_leaf(v) else cond[v]

    _levels(st, condense, root_first=True)
    _levels(st, nest, root_first=False)
    transfer[0] = None
    return explicit, rank, leaf_basis, transfer, svals


def to_h2(h: HValues, st: Structure, eps: float | None = None,
          cond_eps: float | None = None) -> H2Values:
    """Nested row/column bases with transfer matrices and couplings."""
    eps = h.eps if eps is None else eps
    cond_eps = eps / 10.0 if cond_eps is None else cond_eps
    rW, rrank, rleaf, rtr, rsv = _nested_side(st, st.row_blocks(True), h.W, h.sigma, eps, cond_eps)
    cX, crank, cleaf, ctr, csv = _nested_side(st, st.col_blocks(True), h.X, h.sigma, eps, cond_eps)
    coupling = [None] * st.nblocks
    for b in np.nonzero(st.blk_adm)[0]:
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        if h.sigma[b] is None or len(h.sigma[b]) == 0:
            coupling[b] = np.zeros((rrank[t], crank[s]), order="F")
            continue
        L = rW[t].T @ h.W[b]
        R = h.X[b].T @ cX[s]
        coupling[b] = np.asfortranarray((L * h.sigma[b][None, :]) @ R)
    return H2Values(h.kernel, eps, list(h.dense), rrank, crank, rleaf, rtr, cleaf, ctr,
                    rsv, csv, coupling)
