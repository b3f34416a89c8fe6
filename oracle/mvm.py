"""Oracle: the hierarchical matrix-vector product y := alpha*M*x + y (eq. 4).

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

The product of a stored hierarchical matrix has a plain definition: the sum
over all block leaves b = (tau, sigma) of the stored block applied to x|sigma
and added to y|tau.  Every function here writes that definition out, in
float64, with numpy matrix-vector products as the only library primitive.
Vectors at this interface are in original point order; internally they are
permuted to cluster order (perm[i] = original index of cluster position i).

* H (Sec. 3.1): dense leaf y|t += a D x|s, low-rank leaf
  y|t += a U (V^T x|s) with U = W diag(sigma), V = X.  Three evaluation
  orders are provided: block order (eq. 4 summed block by block), leaf-row
  order (each output row cluster rho sums the rows of rho of every block
  whose row cluster contains it; the leaves of the cluster tree partition
  the rows, so every row is summed exactly once) and expansion to a dense
  matrix (small n only).
* UH (Sec. 3.2): forward transformation s_s = X_s^T x|s for every column
  cluster (Alg. 4), coupling sums t_t = sum S_ts s_s over the low-rank blocks
  of each block row (eq. 5), backward transformation y|t += a W_t t_t and the
  dense leaves (Alg. 5).
* H^2 (Sec. 3.3): upward pass s = X^T x|s at leaves and s_s = sum over sons
  s' of F_s'^T s_s' above (Alg. 6), coupling sums, downward pass
  t_t' += E_t' t_t from the root to the leaves, y|t += a W_t t_t at leaves,
  plus the dense leaves (Alg. 7).  In Alg. 7 the coupling of t' happens before
  its parent pushes coefficients down, so the push is an accumulation.

The real-valued data makes every conjugate transpose a plain transpose.
"""
from __future__ import annotations

import numpy as np

from synth.inputs import Structure


def _to_cluster(st: Structure, v: np.ndarray) -> np.ndarray:
    return np.asarray(v, dtype=np.float64)[st.perm]


def _from_cluster(st: Structure, vc: np.ndarray) -> np.ndarray:
    out = np.empty_like(vc)
    out[st.perm] = vc
    return out


def _seg(st: Structure, v: int):
    return slice(int(st.begin[v]), int(st.end[v]))


def _leaves(st: Structure):
    return [v for v in range(st.nnodes) if st.is_leaf(v)]


# ----------------------------------------------------------------------------- H

def h_mvm(st: Structure, dense, W, sigma, X, alpha: float, x: np.ndarray, y: np.ndarray,
          order: str = "block") -> np.ndarray:
    """y + alpha*M*x for an H-matrix given per block (dense | W, sigma, X)."""
    xc = _to_cluster(st, x)
    yc = _to_cluster(st, y).copy()

    def apply(b):
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        if st.blk_adm[b]:
            if sigma[b] is None or len(sigma[b]) == 0:
                return
            tb = X[b].T @ xc[_seg(st, s)]
            yc[_seg(st, t)] += alpha * (W[b] @ (sigma[b] * tb))
        else:
            yc[_seg(st, t)] += alpha * (dense[b] @ xc[_seg(st, s)])

    if order == "block":                      # eq. 4, one block after the other
        for b in range(st.nblocks):
            apply(b)
    elif order == "rows":                     # per leaf row cluster rho
        for rho in _leaves(st):
            r0, r1 = int(st.begin[rho]), int(st.end[rho])
            acc = np.zeros(r1 - r0)
            for b in range(st.nblocks):
                t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
                if not (st.begin[t] <= r0 and r1 <= st.end[t]):
                    continue
                rows = slice(r0 - int(st.begin[t]), r1 - int(st.begin[t]))
                if st.blk_adm[b]:
                    if sigma[b] is not None and len(sigma[b]):
                        acc += W[b][rows] @ (sigma[b] * (X[b].T @ xc[_seg(st, s)]))
                else:
                    acc += dense[b][rows] @ xc[_seg(st, s)]
            yc[r0:r1] += alpha * acc
    elif order == "dense":
        M = h_to_dense(st, dense, W, sigma, X)
        yc += alpha * (M @ xc)
    else:
        raise ValueError(order)
    return _from_cluster(st, yc)


def h_to_dense(st: Structure, dense, W, sigma, X) -> np.ndarray:
    """The stored H-matrix expanded to a dense matrix in cluster order."""
    M = np.zeros((st.n, st.n))
    for b in range(st.nblocks):
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        if st.blk_adm[b]:
            if sigma[b] is not None and len(sigma[b]):
                M[_seg(st, t), _seg(st, s)] = (W[b] * sigma[b][None, :]) @ X[b].T
        else:
            M[_seg(st, t), _seg(st, s)] = dense[b]
    return M


# ---------------------------------------------------------------------------- UH

def uh_mvm(st: Structure, dense, row_basis, col_basis, coupling, alpha: float,
           x: np.ndarray, y: np.ndarray, order: str = "phases") -> np.ndarray:
    xc = _to_cluster(st, x)
    yc = _to_cluster(st, y).copy()
    if order == "dense":
        M = uh_to_dense(st, dense, row_basis, col_basis, coupling)
        return _from_cluster(st, yc + alpha * (M @ xc))
    # Alg. 4: forward transformation for every column cluster
    s = [col_basis[v].T @ xc[_seg(st, v)] for v in range(st.nnodes)]
    rows_lr = st.row_blocks(True)
    rows_d = st.row_blocks(False)
    if order == "phases":
        for t in range(st.nnodes):
            tt = np.zeros(row_basis[t].shape[1])
            for b in rows_lr.get(t, []):            # eq. 5
                tt += coupling[b] @ s[int(st.blk_sigma[b])]
            yc[_seg(st, t)] += alpha * (row_basis[t] @ tt)
        for b in range(st.nblocks):
            if not st.blk_adm[b]:
                yc[_seg(st, int(st.blk_tau[b]))] += alpha * (dense[b] @ xc[_seg(st, int(st.blk_sigma[b]))])
    elif order == "rows":                           # per leaf row cluster rho
        # t_tau by eq. 5 for every row cluster, then y|rho sums, over every
        # tau containing rho, the rows of rho of W_tau t_tau and of the dense
        # blocks of tau's block row
        tt = [np.zeros(row_basis[t].shape[1]) for t in range(st.nnodes)]
        for b in range(st.nblocks):
            if st.blk_adm[b]:
                tt[int(st.blk_tau[b])] += coupling[b] @ s[int(st.blk_sigma[b])]
        for rho in _leaves(st):
            r0, r1 = int(st.begin[rho]), int(st.end[rho])
            acc = np.zeros(r1 - r0)
            for t in range(st.nnodes):
                if not (st.begin[t] <= r0 and r1 <= st.end[t]):
                    continue
                rows = slice(r0 - int(st.begin[t]), r1 - int(st.begin[t]))
                acc += row_basis[t][rows] @ tt[t]
                for b in rows_d.get(t, []):
                    acc += dense[b][rows] @ xc[_seg(st, int(st.blk_sigma[b]))]
            yc[r0:r1] += alpha * acc
    else:
        raise ValueError(order)
    return _from_cluster(st, yc)


def uh_to_dense(st: Structure, dense, row_basis, col_basis, coupling) -> np.ndarray:
    M = np.zeros((st.n, st.n))
    for b in range(st.nblocks):
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        if st.blk_adm[b]:
            M[_seg(st, t), _seg(st, s)] = row_basis[t] @ coupling[b] @ col_basis[s].T
        else:
            M[_seg(st, t), _seg(st, s)] = dense[b]
    return M


# ---------------------------------------------------------------------------- H2

def h2_explicit_bases(st: Structure, leaf_basis, transfer):
    """Explicit cluster bases from the nested representation (Sec. 2.4):
    W_t = [W_t0 E_t0 ; W_t1 E_t1] above the leaves."""
    N = st.nnodes
    out = [None] * N
    for v in np.argsort(-st.level, kind="stable"):
        v = int(v)
        if st.is_leaf(v):
            out[v] = leaf_basis[v]
        else:
            a, b = st.sons(v)
            out[v] = np.vstack([out[a] @ transfer[a], out[b] @ transfer[b]])
    return out


def h2_mvm(st: Structure, dense, row_rank, col_rank, row_leaf_basis, row_transfer,
           col_leaf_basis, col_transfer, coupling, alpha: float, x: np.ndarray,
           y: np.ndarray, order: str = "phases") -> np.ndarray:
    xc = _to_cluster(st, x)
    yc = _to_cluster(st, y).copy()
    N = st.nnodes
    if order == "via_uh":
        rb = h2_explicit_bases(st, row_leaf_basis, row_transfer)
        cb = h2_explicit_bases(st, col_leaf_basis, col_transfer)
        return uh_mvm(st, dense, rb, cb, coupling, alpha, x, y, order="phases")
    # Alg. 6: upward pass, leaves to root
    s = [None] * N
    for v in np.argsort(-st.level, kind="stable"):
        v = int(v)
        if st.is_leaf(v):
            s[v] = col_leaf_basis[v].T @ xc[_seg(st, v)]
        else:
            acc = np.zeros(int(col_rank[v]))
            for c in st.sons(v):
                acc += col_transfer[c].T @ s[c]
            s[v] = acc
    # eq. 5: coupling sums per block row
    rows_lr = st.row_blocks(True)
    t = [np.zeros(int(row_rank[v])) for v in range(N)]
    for v in range(N):
        for b in rows_lr.get(v, []):
            t[v] += coupling[b] @ s[int(st.blk_sigma[b])]
    # downward pass, root to leaves; y updated at the leaves only
    for v in np.argsort(st.level, kind="stable"):
        v = int(v)
        if st.is_leaf(v):
            yc[_seg(st, v)] += alpha * (row_leaf_basis[v] @ t[v])
        else:
            for c in st.sons(v):
                t[c] = t[c] + row_transfer[c] @ t[v]
    for b in range(st.nblocks):
        if not st.blk_adm[b]:
            yc[_seg(st, int(st.blk_tau[b]))] += alpha * (dense[b] @ xc[_seg(st, int(st.blk_sigma[b]))])
    return _from_cluster(st, yc)


# ------------------------------------------------------------------- many RHS

def columns(fn, X: np.ndarray, Y: np.ndarray, *args, **kw) -> np.ndarray:
    """Many right-hand sides: column j of the result is the single-vector
    product applied to X[:, j] and Y[:, j]."""
    out = np.empty_like(np.asarray(Y, dtype=np.float64))
    for j in range(X.shape[1]):
        out[:, j] = fn(*args, x=X[:, j], y=Y[:, j], **kw)
    return out
