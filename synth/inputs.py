"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds none of the matrix-vector product's arithmetic: only points, kernels,
right-hand sides and the neutral description of a block partition that the
compressors below consume.

The paper's matrix is a Galerkin BEM discretisation of the Laplace single
layer potential on the unit sphere (Sec. 2.1, eq. 1-2).  Triangulation and
quadrature are not available here, so point kernels on random sphere points
stand in for it:

* points: normalised Gaussian triples (uniform on the unit sphere),
* Laplace kernel 1/(4 pi |x-y|) and the screened kernel exp(-|x-y|)/|x-y|,
  both with a zero diagonal.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

KERNEL_LAPLACE = 0
KERNEL_EXPR = 1
KERNEL_CONST = 2      # test kernel: 1 off the diagonal
KERNEL_IDENTITY = 3   # test kernel: delta_ij
KERNEL_RANK1 = 4      # test kernel: f(x) g(y) off the diagonal

KERNEL_NAMES = {
    "laplace": KERNEL_LAPLACE,
    "expr": KERNEL_EXPR,
    "const": KERNEL_CONST,
    "identity": KERNEL_IDENTITY,
    "rank1": KERNEL_RANK1,
}


def sphere_points(n: int, seed: int) -> np.ndarray:
    """n x 3 FP64 points uniform on the unit sphere (normalised Gaussians)."""
    g = np.random.default_rng(seed).standard_normal((n, 3))
    return g / np.sqrt((g * g).sum(axis=1))[:, None]


def gaussian_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n)


def gaussian_matrix(n: int, r: int, seed: int) -> np.ndarray:
    """n x r column-major (Fortran order) N(0,1) block of right-hand sides."""
    return np.asfortranarray(np.random.default_rng(seed).standard_normal((n, r)))


def rank1_factors(p: np.ndarray):
    """f(p) = 1 + p_x, g(p) = 2 + p_y p_z for the rank-1 test kernel."""
    return 1.0 + p[:, 0], 2.0 + p[:, 1] * p[:, 2]


def kernel_block(kind: int, prow: np.ndarray, pcol: np.ndarray,
                 grow: np.ndarray, gcol: np.ndarray) -> np.ndarray:
    """Dense kernel block K[a, b] = k(prow[a], pcol[b]), zero where the
    global indices grow[a] == gcol[b] (the diagonal).  Column-major output."""
    same = grow[:, None] == gcol[None, :]
    if kind == KERNEL_IDENTITY:
        return np.asfortranarray(same.astype(np.float64))
    if kind == KERNEL_CONST:
        out = np.ones((len(prow), len(pcol)))
    elif kind == KERNEL_RANK1:
        f, _ = rank1_factors(prow)
        _, g = rank1_factors(pcol)
        out = f[:, None] * g[None, :]
    else:
        d = prow[:, None, :] - pcol[None, :, :]
        r = np.sqrt((d * d).sum(axis=2))
        with np.errstate(divide="ignore", invalid="ignore"):
            if kind == KERNEL_LAPLACE:
                out = 1.0 / (4.0 * np.pi * r)
            elif kind == KERNEL_EXPR:
                out = np.exp(-r) / r
            else:
                raise ValueError(f"unknown kernel {kind}")
    out[same] = 0.0
    return np.asfortranarray(out)


@dataclass
class Structure:
    """Neutral description of a cluster tree and block tree.

    Positions refer to cluster order: perm[i] is the original index of the
    point at cluster position i.  Node tau covers positions
    [begin[tau], end[tau]).  Trees are binary (son0/son1 = -1 at leaves).
    Blocks are pairs of node ids with an admissibility flag.
    """
    n: int
    perm: np.ndarray
    begin: np.ndarray
    end: np.ndarray
    level: np.ndarray
    parent: np.ndarray
    son0: np.ndarray
    son1: np.ndarray
    blk_tau: np.ndarray
    blk_sigma: np.ndarray
    blk_adm: np.ndarray
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def nnodes(self) -> int:
        return len(self.begin)

    @property
    def nblocks(self) -> int:
        return len(self.blk_tau)

    def size(self, v: int) -> int:
        return int(self.end[v] - self.begin[v])

    def is_leaf(self, v: int) -> bool:
        return self.son0[v] < 0

    def sons(self, v: int):
        return [] if self.son0[v] < 0 else [int(self.son0[v]), int(self.son1[v])]

    def row_blocks(self, lowrank: bool | None = None):
        """dict node -> list of block ids whose row cluster is that node."""
        key = ("row", lowrank)
        if key not in self._cache:
            d: dict[int, list[int]] = {}
            for b in range(self.nblocks):
                if lowrank is None or bool(self.blk_adm[b]) == lowrank:
                    d.setdefault(int(self.blk_tau[b]), []).append(b)
            self._cache[key] = d
        return self._cache[key]

    def col_blocks(self, lowrank: bool | None = None):
        key = ("col", lowrank)
        if key not in self._cache:
            d: dict[int, list[int]] = {}
            for b in range(self.nblocks):
                if lowrank is None or bool(self.blk_adm[b]) == lowrank:
                    d.setdefault(int(self.blk_sigma[b]), []).append(b)
            self._cache[key] = d
        return self._cache[key]

    def leaves(self):
        return [v for v in range(self.nnodes) if self.son0[v] < 0]

    def max_level(self) -> int:
        return int(self.level.max())

    def block_coords(self) -> np.ndarray:
        """nb x 4 int64 array (row0, nrows, col0, ncols) in cluster positions."""
        t, s = self.blk_tau, self.blk_sigma
        return np.stack([self.begin[t], self.end[t] - self.begin[t],
                         self.begin[s], self.end[s] - self.begin[s]], axis=1).astype(np.int64)
