"""Oracle: cluster tree, block tree and partition validator.

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

Cluster tree (Def. 2.1): a binary tree of disjoint index sets whose root is
I; every inner node is the disjoint union of its sons; level = distance from
the root.  The paper names no clustering rule, so geometric bisection is used:

* the bounding box of a cluster is the tight axis-aligned box of its points;
* a cluster with at most `leaf_size` points is a leaf;
* otherwise split along the axis of largest extent (lowest axis on ties) at
  the box midpoint 0.5*(lo+hi): son 0 takes the points with coordinate < mid,
  son 1 the rest, both keeping their relative order; if a side is empty the
  cluster is split at half its size instead;
* the permutation lists leaves in depth-first order (son 0 first).

Block tree (Def. 2.2): starting at (I, I), a block is a leaf if it is
admissible or either cluster is a leaf; otherwise its sons are all pairs of
sons (tau-son major).  Admissibility (only named in the paper, Sec. 2.2) is
the standard one on bounding boxes with eta = 2: min(diam) <= 2 dist, taken
on squared quantities with dist > 0:

    diam^2 = sum_d (hi_d - lo_d)^2,
    dist^2 = sum_d max(0, lo_s,d - hi_t,d, lo_t,d - hi_s,d)^2,
    adm    = min(diam_t^2, diam_s^2) <= 4 dist^2  and  dist^2 > 0.

Sums run over x, y, z in that order in plain float64.

Other partitions (the remark after Def. 2.3: BLR and HODLR belong to the same
set of matrices through the choice of clustering and admissibility alone):

* balanced clustering, used by both: every cluster above a fixed depth d
  splits along the axis of largest box extent (lowest axis on ties) into the
  first floor(m/2) of its points ordered by that coordinate (stable order on
  ties) and the rest; d is the smallest depth with ceil(n / 2^d) <= leaf_size,
  and a single point is always a leaf;
* HODLR: off-diagonal admissibility, every block (tau, sigma) with
  tau != sigma is low rank;
* BLR: a single hierarchy level, the block tree recurses to the pairs of leaf
  clusters, which are low rank where the standard condition holds.
"""
from __future__ import annotations

import numpy as np

from synth.inputs import Structure


STANDARD, HODLR, BLR = "standard", "hodlr", "blr"


def balanced_depth(n: int, leaf_size: int) -> int:
    d = 0
    while -(-n // (1 << d)) > leaf_size:
        d += 1
    return d


def cluster_tree(points: np.ndarray, leaf_size: int = 64, balanced: bool = False):
    """Returns (perm, begin, end, level, parent, son0, son1, lo, hi)."""
    n = points.shape[0]
    depth = balanced_depth(n, leaf_size) if balanced else None
    P = np.asarray(points, dtype=np.float64)
    perm = np.empty(n, dtype=np.int64)
    begin, end, level, parent, son0, son1, lo_l, hi_l = [], [], [], [], [], [], [], []
    pos = [0]

    def new_node(lvl, par):
        for lst, val in ((begin, 0), (end, 0), (level, lvl), (parent, par), (son0, -1),
                         (son1, -1), (lo_l, None), (hi_l, None)):
            lst.append(val)
        return len(begin) - 1

    # explicit stack to avoid deep Python recursion: (idx, level, parent, slot)
    root = new_node(0, -1)
    stack = [(np.arange(n, dtype=np.int64), root)]
    while stack:
        idx, v = stack.pop()
        pts = P[idx]
        lo = pts.min(axis=0) if len(idx) else np.zeros(3)
        hi = pts.max(axis=0) if len(idx) else np.zeros(3)
        lo_l[v], hi_l[v] = lo, hi
        leaf = (level[v] >= depth or len(idx) < 2) if balanced else len(idx) <= leaf_size
        if leaf:
            begin[v] = pos[0]
            perm[pos[0]:pos[0] + len(idx)] = idx
            pos[0] += len(idx)
            end[v] = pos[0]
            continue
        ext = hi - lo
        axis = int(np.argmax(ext))          # first maximum on ties
        if balanced:
            srt = idx[np.argsort(pts[:, axis], kind="stable")]
            h = len(idx) // 2
            a, b = srt[:h], srt[h:]
        else:
            mid = 0.5 * (lo[axis] + hi[axis])
            mask = pts[:, axis] < mid
            a, b = idx[mask], idx[~mask]
            if len(a) == 0 or len(b) == 0:
                h = len(idx) // 2
                a, b = idx[:h], idx[h:]
        c0 = new_node(level[v] + 1, v)
        c1 = new_node(level[v] + 1, v)
        son0[v], son1[v] = c0, c1
        begin[v] = -1  # filled after sons
        # depth-first, son 0 first: push son 1 below son 0
        stack.append((b, c1))
        stack.append((a, c0))
    # node ids above are in creation order; renumber to depth-first pre-order
    N = len(begin)
    order = []
    st = [0]
    while st:
        v = st.pop()
        order.append(v)
        if son0[v] >= 0:
            st.append(son1[v])
            st.append(son0[v])
    newid = np.empty(N, dtype=np.int64)
    newid[np.array(order)] = np.arange(N)
    def remap(lst):
        return np.array([lst[v] for v in order], dtype=np.int64)
    son0_a = np.array([newid[son0[v]] if son0[v] >= 0 else -1 for v in order], dtype=np.int64)
    son1_a = np.array([newid[son1[v]] if son1[v] >= 0 else -1 for v in order], dtype=np.int64)
    par_a = np.array([newid[parent[v]] if parent[v] >= 0 else -1 for v in order], dtype=np.int64)
    lev_a = remap(level)
    lo_a = np.array([lo_l[v] for v in order])
    hi_a = np.array([hi_l[v] for v in order])
    beg_a = remap(begin)
    end_a = remap(end)
    # inner nodes: [begin of son0, end of son1), computed bottom-up
    for v in range(N - 1, -1, -1):
        if son0_a[v] >= 0:
            beg_a[v] = beg_a[son0_a[v]]
            end_a[v] = end_a[son1_a[v]]
    return perm, beg_a, end_a, lev_a, par_a, son0_a, son1_a, lo_a, hi_a


def admissible(lo_t, hi_t, lo_s, hi_s) -> bool:
    """Standard admissibility min(diam) <= 2 dist on bounding boxes."""
    dt = 0.0
    ds = 0.0
    dd = 0.0
    for d in range(3):
        et = float(hi_t[d]) - float(lo_t[d])
        es = float(hi_s[d]) - float(lo_s[d])
        dt = dt + et * et
        ds = ds + es * es
        g = 0.0
        a = float(lo_s[d]) - float(hi_t[d])
        b = float(lo_t[d]) - float(hi_s[d])
        if a > g:
            g = a
        if b > g:
            g = b
        dd = dd + g * g
    return (min(dt, ds) <= 4.0 * dd) and dd > 0.0


def partition_admissible(kind, t, s, son0, lo, hi) -> bool:
    """The admissibility of the chosen partition kind."""
    if kind == HODLR:
        return t != s
    if kind == BLR:
        return son0[t] < 0 and son0[s] < 0 and admissible(lo[t], hi[t], lo[s], hi[s])
    return admissible(lo[t], hi[t], lo[s], hi[s])


def block_tree(son0, son1, lo, hi, kind=STANDARD):
    """Leaves of the block tree in depth-first order: (tau, sigma, adm)."""
    taus, sigs, adms = [], [], []
    stack = [(0, 0)]
    while stack:
        t, s = stack.pop()
        if partition_admissible(kind, t, s, son0, lo, hi):
            taus.append(t); sigs.append(s); adms.append(True)
        elif son0[t] < 0 or son0[s] < 0:
            taus.append(t); sigs.append(s); adms.append(False)
        else:
            pairs = [(int(son0[t]), int(son0[s])), (int(son0[t]), int(son1[s])),
                     (int(son1[t]), int(son0[s])), (int(son1[t]), int(son1[s]))]
            for p in reversed(pairs):
                stack.append(p)
    return (np.array(taus, dtype=np.int64), np.array(sigs, dtype=np.int64),
            np.array(adms, dtype=bool))


def build_structure(points: np.ndarray, leaf_size: int = 64, kind: str = STANDARD) -> Structure:
    perm, beg, end, lev, par, s0, s1, lo, hi = cluster_tree(points, leaf_size, balanced=kind != STANDARD)
    bt, bs, ba = block_tree(s0, s1, lo, hi, kind)
    st = Structure(points.shape[0], perm, beg, end, lev, par, s0, s1, bt, bs, ba)
    st._cache["bbox"] = (lo, hi)
    st._cache["partition"] = kind
    return st


def validate_partition(st: Structure, leaf_size: int = 64) -> None:
    """Raises AssertionError unless the block leaves partition I x I exactly
    once, every low-rank leaf is admissible, every dense leaf has a leaf
    cluster, blocks pair clusters of equal level, and sons partition their
    parent (Def. 2.1, 2.2)."""
    n = st.n
    kind = st._cache.get("partition", STANDARD)
    assert sorted(st.perm.tolist()) == list(range(n)), "perm is not a permutation"
    for v in range(st.nnodes):
        if st.son0[v] >= 0:
            a, b = int(st.son0[v]), int(st.son1[v])
            assert st.begin[a] == st.begin[v] and st.end[a] == st.begin[b] and st.end[b] == st.end[v]
            assert st.level[a] == st.level[v] + 1 == st.level[b]
            assert st.end[a] > st.begin[a] and st.end[b] > st.begin[b]
        else:
            assert 0 < st.end[v] - st.begin[v] <= leaf_size or n == 0
            if kind != STANDARD and st.end[v] - st.begin[v] > 1:
                assert st.level[v] == balanced_depth(n, leaf_size)
    lo, hi = st._cache.get("bbox", (None, None))
    kind = st._cache.get("partition", STANDARD)
    for b in range(st.nblocks):
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        assert st.level[t] == st.level[s]
        if st.blk_adm[b]:
            if lo is not None:
                assert partition_admissible(kind, t, s, st.son0, lo, hi)
        else:
            assert st.son0[t] < 0 or st.son0[s] < 0
    # exact cover: per leaf row cluster, the column intervals of every block
    # whose row cluster contains it must tile [0, n) without gap or overlap
    total = 0
    for b in range(st.nblocks):
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        total += int(st.end[t] - st.begin[t]) * int(st.end[s] - st.begin[s])
    assert total == n * n, f"block areas sum to {total}, not n^2={n * n}"
    leaves = [v for v in range(st.nnodes) if st.son0[v] < 0]
    anc_blocks: dict[int, list] = {}
    for b in range(st.nblocks):
        anc_blocks.setdefault(int(st.blk_tau[b]), []).append(b)
    for rho in leaves:
        ivs = []
        v = rho
        while v >= 0:
            for b in anc_blocks.get(v, []):
                s = int(st.blk_sigma[b])
                ivs.append((int(st.begin[s]), int(st.end[s])))
            v = int(st.parent[v])
        ivs.sort()
        pos = 0
        for a, e in ivs:
            assert a == pos, f"gap/overlap in block row of leaf {rho} at {pos}"
            pos = e
        assert pos == n


def coverage_bitmap(st: Structure) -> np.ndarray:
    """n x n count of how many block leaves cover each index pair (brute force)."""
    cnt = np.zeros((st.n, st.n), dtype=np.int32)
    for b in range(st.nblocks):
        t, s = int(st.blk_tau[b]), int(st.blk_sigma[b])
        cnt[st.begin[t]:st.end[t], st.begin[s]:st.end[s]] += 1
    return cnt
