"""The C-ABI library loads, exports every declared symbol, and its host-side
tree builder matches the oracle bit-exactly (no GPU needed)."""
import os
import re

import numpy as np
import pytest

from oracle import build_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lrsp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lrsp_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1811_11248_amd import lrsp
    return lrsp


def test_library_exports_every_declared_symbol(L):
    h = L.lib()
    names = _declared()
    assert "lrsp_factor" in names and "lrsp_pcg" in names
    for name in names:
        assert hasattr(h, name), name
    bound = {n for n, _, _ in L.SIGNATURES}
    assert set(names) <= bound


@pytest.mark.parametrize("grid,leaf", [
    ((64, 64, 1, 1), 64), ((64, 64, 16, 1), 256), ((128, 128, 20, 2), 256),
    ((13, 11, 5, 1), 40), ((5, 3, 2, 1), 8), ((17, 17, 8, 1), 256), ((48, 31, 9, 2), 100),
    ((7, 3, 4, 1), 1000)])
def test_tree_matches_oracle(L, grid, leaf):
    e = L.Tree(grid, leaf).export()
    o = build_tree(grid, leaf)
    assert e["nlevels"] == o.nlevels
    assert len(e["leaf_dofs"]) == len(o.leaf_dofs)
    for a, b in zip(e["leaf_dofs"], o.leaf_dofs):
        assert np.array_equal(a, b)


def test_tree_errors(L):
    with pytest.raises(L.LrspError) as ex:
        L.Tree((4, 4, 8, 1), 4)
    assert ex.value.status == L.ERR_ARG
    with pytest.raises(L.LrspError):
        L.Tree((1, 1, 8, 2), 15)
