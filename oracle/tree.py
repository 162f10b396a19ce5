"""Cluster tree and level schedule of the oracle.

The paper clusters the unknowns with a geometric partitioner (Zoltan, clusters
of about 100 DoFs) applied to ONE horizontal layer of the extruded mesh and
then extrudes the partition, so that every vertical line of mesh vertices lies
in one cluster (section "Extruded Partitioning for Ice Sheets").  Coarser
levels have half as many clusters as the level below (discussion of the
per-level time breakdown in the Numerical Results section).

Reading used here (the paper does not fix the partitioner's rule):

* the horizontal index box ``[0,nx) x [0,ny)`` is bisected recursively
  exactly ``L`` times, ``L`` the smallest integer with ``leaf * 2**L >= N``;
* each split halves the longer side (ties: the x side) at
  ``mid = lo + len // 2``; the left child is ``[lo, mid)``;
* level-0 clusters are the depth-``L`` boxes in left-to-right (depth-first)
  order and a cluster's DoFs are sorted by global id; the level-``l``
  cluster ``c`` is the parent of level-``(l-1)`` clusters ``2c`` and ``2c+1``.

Two clusters are neighbours when their block of the current matrix is
structurally nonzero (section "Scaled Low-rank Elimination").
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class ClusterTree:
    grid: tuple
    leaf: int
    nlevels: int  # L: number of bisections (level-0 clusters = 2**L)
    boxes: list  # boxes[d] = list of (x0, x1, y0, y1) at depth d
    leaf_dofs: list  # level-0 cluster DoF lists (sorted global ids)

    @property
    def nleaves(self) -> int:
        return len(self.leaf_dofs)

    def perm(self) -> np.ndarray:
        """Level-0 cluster order of the global DoFs (concatenated leaf lists)."""
        return np.concatenate(self.leaf_dofs) if self.leaf_dofs else np.zeros(0, np.int64)

    def dof_cluster(self) -> np.ndarray:
        n = sum(len(d) for d in self.leaf_dofs)
        cl = np.empty(n, np.int64)
        for c, d in enumerate(self.leaf_dofs):
            cl[d] = c
        return cl


def num_levels(n: int, leaf: int) -> int:
    L = 0
    while leaf * (1 << L) < n:
        L += 1
    return L


def build_tree(grid, leaf: int) -> ClusterTree:
    nx, ny, nz, nc = (int(v) for v in grid)
    if leaf < nz * nc:
        raise ValueError("leaf size smaller than one vertical column")
    n = nx * ny * nz * nc
    L = num_levels(n, leaf)
    boxes = [[(0, nx, 0, ny)]]
    for _ in range(L):
        nxt = []
        for (x0, x1, y0, y1) in boxes[-1]:
            lx, ly = x1 - x0, y1 - y0
            if lx >= ly:
                if lx < 2:
                    raise ValueError("a box would have to split a single column")
                mid = x0 + lx // 2
                nxt += [(x0, mid, y0, y1), (mid, x1, y0, y1)]
            else:
                mid = y0 + ly // 2
                nxt += [(x0, x1, y0, mid), (x0, x1, mid, y1)]
        boxes.append(nxt)
    col = nz * nc
    leaf_dofs = []
    for (x0, x1, y0, y1) in boxes[-1]:
        ids = []
        for y in range(y0, y1):
            for x in range(x0, x1):
                base = col * (x + nx * y)
                ids.extend(range(base, base + col))
        leaf_dofs.append(np.array(sorted(ids), dtype=np.int64))
    return ClusterTree((nx, ny, nz, nc), leaf, L, boxes, leaf_dofs)


def level0_graph(tree: ClusterTree, rowptr, col) -> list:
    """Clusters p != q are neighbours iff A has a stored entry between them."""
    cl = tree.dof_cluster()
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    cp = cl[rows]
    cq = cl[np.asarray(col)]
    mask = cp != cq
    pairs = set(zip(cp[mask].tolist(), cq[mask].tolist()))
    adj = [set() for _ in range(tree.nleaves)]
    for p, q in pairs:
        adj[p].add(q)
        adj[q].add(p)
    return [sorted(a) for a in adj]


def d2_colouring(adj: list) -> list:
    """Greedy distance-2 colouring in index order: each cluster takes the
    smallest colour not used by an already-coloured cluster within two hops."""
    M = len(adj)
    colour = [-1] * M
    for s in range(M):
        near = set(adj[s])
        for q in adj[s]:
            near.update(adj[q])
        near.discard(s)
        used = {colour[q] for q in near if colour[q] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[s] = c
    return colour


def coarsen_square(adj: list) -> list:
    """Graph of the parents (c -> c//2) of all pairs within two hops."""
    M = len(adj)
    P = (M + 1) // 2
    out = [set() for _ in range(P)]
    for s in range(M):
        near = set(adj[s])
        for q in adj[s]:
            near.update(adj[q])
        for q in near:
            if q // 2 != s // 2:
                out[s // 2].add(q // 2)
    return [sorted(a) for a in out]
