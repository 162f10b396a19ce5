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

For unstructured extruded meshes ``build_tree_graph`` partitions the layer
graph instead (level-structure bisection, the graph alone).

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


def _bfs_order(S: list, adj_ptr, adj, start: int) -> tuple:
    """Breadth-first order of the vertex set S (ascending list) from start,
    over the subgraph S induces, neighbours taken in increasing id; when the
    queue empties the search restarts at the smallest unvisited vertex of S.
    Returns (order, distance of each vertex of start's component)."""
    inside = set(S)
    seen = {start}
    order = [start]
    dist = {start: 0}
    head = 0
    first_comp = True
    nxt_unvisited = 0
    while len(order) < len(S):
        if head == len(order):
            # restart at the smallest unvisited vertex (another component)
            while S[nxt_unvisited] in seen:
                nxt_unvisited += 1
            v = S[nxt_unvisited]
            seen.add(v)
            order.append(v)
            first_comp = False
        u = order[head]
        head += 1
        for e in range(adj_ptr[u], adj_ptr[u + 1]):
            w = int(adj[e])
            if w in inside and w not in seen:
                seen.add(w)
                order.append(w)
                if first_comp and u in dist:
                    dist[w] = dist[u] + 1
    return order, dist


def graph_bisect(S: list, adj_ptr, adj) -> tuple:
    """Level-structure bisection of the vertex set S (ascending list): a
    breadth-first search from the smallest vertex finds a far vertex r (the
    largest distance in its component, ties: smallest id); the breadth-first
    order from r is cut in the middle.  Returns (left, right), each
    ascending; left holds the first floor(|S|/2) vertices of that order."""
    _, dist = _bfs_order(S, adj_ptr, adj, S[0])
    far = max(dist.values())
    r = min(v for v, d in dist.items() if d == far)
    order, _ = _bfs_order(S, adj_ptr, adj, r)
    h = len(S) // 2
    return sorted(order[:h]), sorted(order[h:])


def build_tree_graph(adj_ptr, adj, nz: int, nc: int, leaf: int) -> ClusterTree:
    """Extruded partitioning of an unstructured extruded mesh (section
    "Extruded Partitioning for Ice Sheets": partition one layer with a graph
    partitioner, then extrude every part through all layers).

    The layer is the graph of the ``ncols = len(adj_ptr) - 1`` vertical
    columns (CSR, symmetric, sorted, no self loops); global DoF id of
    component c at layer z of column v is ``c + nc (z + nz v)``.  The column
    set is bisected ``L`` times (``L`` as for the grid tree) by
    ``graph_bisect``, which uses the graph only (no coordinates); children
    are ordered left, right and a leaf's DoFs sorted by global id."""
    adj_ptr = np.asarray(adj_ptr, dtype=np.int64)
    adj = np.asarray(adj, dtype=np.int64)
    ncols = len(adj_ptr) - 1
    col = nz * nc
    if leaf < col or ncols < 1:
        raise ValueError("leaf size smaller than one vertical column")
    n = ncols * col
    L = num_levels(n, leaf)
    sets = [list(range(ncols))]
    for _ in range(L):
        nxt = []
        for S in sets:
            if len(S) < 2:
                raise ValueError("a part would have to split a single column")
            left, right = graph_bisect(S, adj_ptr, adj)
            nxt += [left, right]
        sets = nxt
    leaf_dofs = [np.concatenate([np.arange(v * col, (v + 1) * col, dtype=np.int64) for v in S]) for S in sets]
    return ClusterTree((ncols, 1, nz, nc), leaf, L, [], leaf_dofs)


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
