"""Pins of the oracle's cluster tree and level schedule."""
import numpy as np
import pytest

from oracle import build_tree, coarsen_square, d2_colouring, factor, level0_graph
from synth import config, laplace2d, slab_scalar


def test_tree_golden(golden):
    g = golden("tree_5x3x2_leaf8.json")
    T = build_tree(tuple(g["grid"]), g["leaf"])
    assert T.nlevels == g["nlevels"]
    assert [list(b) for b in T.boxes[-1]] == g["boxes"]
    assert [d.tolist() for d in T.leaf_dofs] == g["leaf_dofs"]


@pytest.mark.parametrize("grid,leaf,L,sizes", [
    ((64, 64, 1, 1), 64, 6, {64}),
    ((64, 64, 16, 1), 256, 8, {256}),
    ((128, 128, 20, 2), 256, 12, {160}),
])
def test_tree_sizes(grid, leaf, L, sizes):
    T = build_tree(grid, leaf)
    assert T.nlevels == L and T.nleaves == 2 ** L
    assert {len(d) for d in T.leaf_dofs} == sizes
    n = int(np.prod(grid))
    assert np.array_equal(np.sort(T.perm()), np.arange(n))


def test_tree_keeps_columns_whole():
    grid = (17, 13, 5, 2)
    T = build_tree(grid, 40)
    col = grid[2] * grid[3]
    cl = T.dof_cluster()
    assert np.all(cl.reshape(-1, col) == cl.reshape(-1, col)[:, :1])
    for d in T.leaf_dofs:
        assert np.all(np.diff(d) > 0)


def test_tree_errors():
    with pytest.raises(ValueError):
        build_tree((4, 4, 8, 1), 4)  # leaf smaller than a column
    with pytest.raises(ValueError):
        build_tree((1, 1, 8, 2), 16 - 1)  # would have to split one column


def test_colouring_golden(golden):
    g = golden("colouring_path4.json")
    col = d2_colouring(g["adj"])
    assert col == g["colour"]
    assert sorted(range(4), key=lambda s: (col[s], s)) == g["order"]


def _check_d2(adj, col):
    M = len(adj)
    for s in range(M):
        near = set(adj[s])
        for q in adj[s]:
            near.update(adj[q])
        near.discard(s)
        assert all(col[q] != col[s] for q in near)
        earlier = {col[q] for q in near if q < s}
        assert all(c in earlier for c in range(col[s]))  # greedy: smallest free


def test_colouring_valid_on_grids():
    for pr, leaf in ((config("laplace64"), 64), (laplace2d(32), 16)):
        T = build_tree(pr.grid, leaf)
        adj = level0_graph(T, pr.rowptr, pr.col)
        _check_d2(adj, d2_colouring(adj))
        _check_d2(coarsen_square(adj), d2_colouring(coarsen_square(adj)))


def test_level_graphs_are_coarsened_squares():
    # the oracle derives each level's graph from the blocks actually present;
    # it must equal the parents of all pairs within two hops of the level below
    kap = np.ones((16, 16, 4))
    pr = slab_scalar(16, 16, 4, 1e3, kap)
    T = build_tree(pr.grid, 32)
    F = factor(pr.rowptr, pr.col, pr.val, T, 1e-2)
    graphs = [lv.graph for lv in F.levels] + [F.top_graph]
    assert graphs[0] == level0_graph(T, pr.rowptr, pr.col)
    for g0, g1 in zip(graphs, graphs[1:]):
        assert coarsen_square(g0) == g1
