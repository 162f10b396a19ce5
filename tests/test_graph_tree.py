"""Extruded partitioning of an unstructured layer (graph tree).

The oracle's level-structure bisection against a hand-derived fixture and
against what any extruded partition must satisfy; the C-ABI builder against
the oracle bit for bit (host code, no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import build_tree_graph
from synth import extruded_mesh, layer_mesh


def _grid_graph(nx, ny):
    idx = np.arange(nx * ny).reshape(ny, nx)
    e = np.concatenate([np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], 1),
                        np.stack([idx[:-1].ravel(), idx[1:].ravel()], 1)])
    e = np.concatenate([e, e[:, ::-1]])
    g = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(nx * ny,) * 2).tocsr()
    g.sum_duplicates()
    g.sort_indices()
    return g.indptr.astype(np.int64), g.indices.astype(np.int32)


def _disconnected():
    # two paths 0-2-4 and 1-3-5-6 (interleaved ids) and an isolated 7
    edges = [(0, 2), (2, 4), (1, 3), (3, 5), (5, 6)]
    e = np.array(edges + [(b, a) for a, b in edges])
    g = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(8, 8)).tocsr()
    g.sort_indices()
    return g.indptr.astype(np.int64), g.indices.astype(np.int32)


def test_fixture_path8(golden):
    f = golden("graph_tree_path8.json")
    T = build_tree_graph(f["adj_ptr"], f["adj"], f["nz"], f["ncomp"], f["leaf"])
    assert T.nlevels == f["nlevels"]
    assert [d.tolist() for d in T.leaf_dofs] == f["leaf_dofs"]


GRAPHS = {
    "grid 9x7": lambda: _grid_graph(9, 7),
    "delaunay 300": lambda: layer_mesh(300, seed=4)[1:],
    "disconnected": _disconnected,
}


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("nz,nc,leaf", [(1, 1, 4), (5, 2, 40), (3, 1, 25)])
def test_partition_properties(name, nz, nc, leaf):
    ap, aj = GRAPHS[name]()
    ncols = len(ap) - 1
    col = nz * nc
    if ncols * col <= leaf:
        pytest.skip("single cluster")
    T = build_tree_graph(ap, aj, nz, nc, leaf)
    n = ncols * col
    assert leaf * 2 ** T.nlevels >= n > leaf * 2 ** (T.nlevels - 1)
    allv = np.sort(np.concatenate(T.leaf_dofs))
    assert np.array_equal(allv, np.arange(n))  # a partition of the DoFs
    for d in T.leaf_dofs:
        assert np.all(np.diff(d) > 0)
        cols = np.unique(d // col)
        assert len(d) == len(cols) * col  # whole vertical columns
    # halving at every split: leaf column counts differ by at most one per level
    counts = [len(d) // col for d in T.leaf_dofs]
    assert max(counts) - min(counts) <= T.nlevels


def test_c_abi_builder_matches_oracle():
    from paper_1811_11248_amd import lrsp
    cases = [(GRAPHS["grid 9x7"](), 1, 1, 4), (GRAPHS["delaunay 300"](), 5, 2, 40),
             (GRAPHS["disconnected"](), 3, 1, 5), (layer_mesh(2000, seed=7)[1:], 20, 2, 256)]
    pr = extruded_mesh(500, 8, 1e3, seed=3)
    cases.append(((pr.params["layer_adj_ptr"], pr.params["layer_adj"]), 8, 2, 128))
    for (ap, aj), nz, nc, leaf in cases:
        e = lrsp.Tree.from_graph(ap, aj, nz, nc, leaf).export()
        o = build_tree_graph(ap, aj, nz, nc, leaf)
        assert e["nlevels"] == o.nlevels
        assert len(e["leaf_dofs"]) == len(o.leaf_dofs)
        for a, b in zip(e["leaf_dofs"], o.leaf_dofs):
            assert np.array_equal(a, b)


def test_c_abi_builder_rejects_bad_graphs():
    from paper_1811_11248_amd import lrsp
    ap, aj = _grid_graph(4, 4)
    with pytest.raises(lrsp.LrspError):
        lrsp.Tree.from_graph(ap, aj, 4, 1, 3)  # leaf below one column
    bad = aj.copy()
    bad[0] = 99  # out of range
    with pytest.raises(lrsp.LrspError):
        lrsp.Tree.from_graph(ap, bad, 1, 1, 4)
    bad = aj.copy()
    bad[0] = 0  # self loop of column 0
    with pytest.raises(lrsp.LrspError):
        lrsp.Tree.from_graph(ap, bad, 1, 1, 4)
