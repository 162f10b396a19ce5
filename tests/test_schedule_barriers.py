"""Host-side check of the barrier rules of the persistent level kernels.

One launch per level runs all colours of a level; between two colours it
normally waits at a grid barrier, but it skips that barrier where both
colours are small:

* ``slre_level_kernel`` (elimination) and ``fwd_level_kernel`` /
  ``bwd_level_kernel`` (sweeps of large clusters): item ``i`` of colour ``c``
  runs on workgroup ``(i - cstart[c]) mod G``; two consecutive colours of at
  most one item each are separated by a workgroup barrier only;
* ``sweep_wave_kernel`` (sweeps of small clusters): item ``i`` runs on wave
  ``o mod nw`` of workgroup ``(o mod G nw) div nw``, ``o = i - cstart[c]``;
  consecutive colours of at most one item each by nothing but the wave's own
  program order, colours of at most ``nw`` items each (or a grid of one
  workgroup) by a workgroup barrier.

This test restates those rules and checks, for every level of the benchmark
workloads, the many-systems batch and the test cases, at several grid sizes,
that every pair of steps touching the same data in different colours is
ordered: by a grid barrier between them, or by a workgroup barrier when one
workgroup runs both, or by program order when one wave runs both.  What a
step touches comes from the symbolic elimination of the level (the same rule
as the oracle: the near field is the level-start graph, the far field the
fill created earlier in the level): the elimination of ``s`` reads and writes
the blocks ``(s, q)`` of its near and far field and the Schur targets
``(p, q)``, ``p, q`` in its near field; its sweep reads and writes the vector
segments of ``s`` and its near field.  Same-colour steps run concurrently,
so they must touch disjoint data (the distance-2 colouring's claim).
"""
import numpy as np
import pytest

from oracle import build_tree, level0_graph
from oracle.tree import coarsen_square, d2_colouring
from synth import batch_params, config, laplace2d, lognormal_field, slab_scalar, slab_vector

NW = 512 // 64  # waves per workgroup of sweep_wave_kernel
GRIDS = (1, 2, 3, 7, 64, 256, 1 << 20)


def _box_graph(tree):
    """Level-0 graph of a box tree: leaves whose boxes share a face segment
    (the 5- and 7-point stencils couple face neighbours only)."""
    boxes = tree.boxes[-1]
    M = len(boxes)
    by_x0, by_y0 = {}, {}
    for p, (x0, x1, y0, y1) in enumerate(boxes):
        by_x0.setdefault(x0, []).append(p)
        by_y0.setdefault(y0, []).append(p)
    adj = [set() for _ in range(M)]
    for p, (x0, x1, y0, y1) in enumerate(boxes):
        for q in by_x0.get(x1, []):  # q to the right of p
            u0, u1, v0, v1 = boxes[q]
            if min(y1, v1) > max(y0, v0):
                adj[p].add(q)
                adj[q].add(p)
        for q in by_y0.get(y1, []):  # q above p
            u0, u1, v0, v1 = boxes[q]
            if min(x1, u1) > max(x0, u0):
                adj[p].add(q)
                adj[q].add(p)
    return [sorted(a) for a in adj]


def _levels(graph):
    """(graph, colour lists, per-cluster factor blocks and sweep segments)
    of every eliminated level, until the graph is complete or one cluster."""
    out = []
    g = graph
    while True:
        M = len(g)
        if M == 1 or all(len(g[p]) == M - 1 for p in range(M)):
            return out
        colour = d2_colouring(g)
        ncol = max(colour) + 1
        cols = [[s for s in range(M) if colour[s] == c] for c in range(ncol)]
        linked = [set(a) for a in g]
        blocks, segs = {}, {}
        for c in range(ncol):
            for s in cols[c]:
                n = set(g[s])
                w = linked[s] - n
                bl = {(s, s)} | {(min(s, q), max(s, q)) for q in n | w}
                bl |= {(min(p, q), max(p, q)) for p in n for q in n}
                blocks[s] = bl
                segs[s] = {s} | n
            # fill created by the colour's eliminations (same-colour steps are
            # independent, so adding it after the colour is the same)
            for s in cols[c]:
                n = g[s]
                for p in n:
                    for q in n:
                        if p != q:
                            linked[p].add(q)
        out.append((g, cols, blocks, segs))
        g = coarsen_square(g)


def _check_same_colour(cols, touch):
    for cl in cols:
        seen = {}
        for s in cl:
            for x in touch[s]:
                assert x not in seen, f"clusters {seen[x]} and {s} of one colour both touch {x}"
                seen[x] = s


def _pairs(cols, touch, reverse=False):
    """Consecutive touches of the same datum in processing order, as arrays
    (position of the earlier and later colour in processing order, their
    offsets within their colours, the two items) for data touched by steps
    of different colours."""
    seq = list(range(len(cols)))[::-1] if reverse else list(range(len(cols)))
    last = {}
    k0, k1, o0, o1, s0, s1 = [], [], [], [], [], []
    for k, c in enumerate(seq):
        for o, s in enumerate(cols[c]):
            for x in touch[s]:
                prev = last.get(x)
                if prev is not None and prev[0] != k:
                    k0.append(prev[0])
                    o0.append(prev[1])
                    s0.append(prev[2])
                    k1.append(k)
                    o1.append(o)
                    s1.append(s)
                last[x] = (k, o, s)
    return seq, (np.array(k0, dtype=np.int64), np.array(k1, dtype=np.int64), np.array(o0, dtype=np.int64),
                 np.array(o1, dtype=np.int64), s0, s1)


def _check_order(seq, pairs, executor, boundary):
    """executor(o) -> (workgroup, wave) arrays; boundary(c, cn) ->
    'grid'|'wg'|'none' for consecutive colours in processing order."""
    k0, k1, o0, o1, s0, s1 = pairs
    if len(k0) == 0:
        return
    bnd = [boundary(seq[k], seq[k + 1]) for k in range(len(seq) - 1)]
    grid_pre = np.concatenate([[0], np.cumsum([b == "grid" for b in bnd])])
    wg_pre = np.concatenate([[0], np.cumsum([b in ("grid", "wg") for b in bnd])])
    wg0, wv0 = executor(o0)
    wg1, wv1 = executor(o1)
    no_grid = grid_pre[k1] - grid_pre[k0] == 0
    has_wg = wg_pre[k1] - wg_pre[k0] > 0
    bad = no_grid & ((has_wg & (wg0 != wg1)) | (~has_wg & ((wg0 != wg1) | (wv0 != wv1))))
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError(f"{s0[i]} (colour {seq[k0[i]]}) and {s1[i]} (colour {seq[k1[i]]}) touch the same "
                             f"data on (workgroup, wave) {(wg0[i], wv0[i])} and {(wg1[i], wv1[i])} "
                             f"with no barrier that orders them")


def _check_level(cols, blocks, segs):
    _check_same_colour(cols, blocks)
    _check_same_colour(cols, segs)
    sz = [len(cl) for cl in cols]
    pf = _pairs(cols, blocks)
    ps_f = _pairs(cols, segs)
    ps_b = _pairs(cols, segs, reverse=True)
    for G in GRIDS:
        # elimination, and sweeps of large clusters (one workgroup per item)
        def ex_wg(o):
            return o % G, np.zeros_like(o)

        def b_single(c, cn):
            return "wg" if sz[c] <= 1 and sz[cn] <= 1 else "grid"
        for seq, pr in (pf, ps_f, ps_b):
            _check_order(seq, pr, ex_wg, b_single)

        # sweeps of small clusters (one wave per item)
        def ex_wave(o):
            return (o % (G * NW)) // NW, o % NW

        def b_wave(c, cn):
            if sz[c] <= 1 and sz[cn] <= 1:
                return "none"
            if G == 1 or (sz[c] <= NW and sz[cn] <= NW):
                return "wg"
            return "grid"
        for seq, pr in (ps_f, ps_b):
            _check_order(seq, pr, ex_wave, b_wave)


def _merge(systems):
    """Batch: per level index, colour c holds the items of colour c of every
    system still eliminating at that level, system after system; touched data
    carry the system id (systems never share data)."""
    merged = []
    depth = max(len(lv) for lv in systems)
    for li in range(depth):
        cols, blocks, segs = [], {}, {}
        for si, lv in enumerate(systems):
            if li >= len(lv):
                continue
            _, c_s, b_s, g_s = lv[li]
            while len(cols) < len(c_s):
                cols.append([])
            for c, cl in enumerate(c_s):
                for s in cl:
                    cols[c].append((si, s))
                    blocks[(si, s)] = {(si, x) for x in b_s[s]}
                    segs[(si, s)] = {(si, x) for x in g_s[s]}
        merged.append((cols, blocks, segs))
    return merged


@pytest.mark.parametrize("name,leaf", [("laplace64", 64), ("slab64", 256), ("stokes128", 256), ("stokes256", 256)])
def test_benchmark_workloads(name, leaf):
    grids = {"laplace64": (64, 64, 1, 1), "slab64": (64, 64, 16, 1), "stokes128": (128, 128, 20, 2),
             "stokes256": (256, 256, 32, 2)}
    T = build_tree(grids[name], leaf)
    levels = _levels(_box_graph(T))
    assert levels
    for g, cols, blocks, segs in levels:
        _check_level(cols, blocks, segs)


def test_box_graph_is_the_matrix_graph():
    # the face-neighbour graph used above equals the graph of the matrix
    for pr, leaf in ((config("laplace64"), 64), (slab_scalar(24, 20, 8, 1e4), 64), (slab_vector(13, 11, 6, 1e3), 120)):
        T = build_tree(pr.grid, leaf)
        assert _box_graph(T) == level0_graph(T, pr.rowptr, pr.col)


def test_many_systems_batch():
    P = batch_params()
    systems = []
    for p in P:
        T = build_tree((p["nx"], p["ny"], p["nz"], 1), 256)
        systems.append(_levels(_box_graph(T)))
    for cols, blocks, segs in _merge(systems):
        _check_level(cols, blocks, segs)


def test_parity_cases():
    cases = [(laplace2d(16), 16), (slab_scalar(13, 11, 5, 1e3, lognormal_field((11, 13, 5), seed=2)), 40),
             (slab_vector(10, 9, 4, 1e2), 48), (slab_scalar(24, 20, 8, 1e4), 64), (laplace2d(32, 2), 16),
             (slab_scalar(24, 20, 8, 1e4), 128), (slab_vector(13, 11, 6, 1e3), 120),
             (slab_scalar(12, 10, 6, 1e4), 48)]
    for pr, leaf in cases:
        T = build_tree(pr.grid, leaf)
        for g, cols, blocks, segs in _levels(level0_graph(T, pr.rowptr, pr.col)):
            _check_level(cols, blocks, segs)


def test_checker_catches_a_missing_barrier():
    # two colours touching one datum, the later item on another workgroup
    # (or wave) with only a workgroup barrier (or none) between them must be
    # reported; a grid barrier, or the same workgroup (wave), orders them
    cols = [[0, 5], [1], [2, 3]]
    touch = {0: {"w"}, 5: {"x"}, 1: {"x"}, 2: {"y"}, 3: {"z"}}
    seq, pr = _pairs(cols, touch)
    with pytest.raises(AssertionError):
        _check_order(seq, pr, lambda o: (o % 2, 0 * o), lambda c, cn: "wg")  # item 5 on wg 1, item 1 on wg 0
    _check_order(seq, pr, lambda o: (o % 2, 0 * o), lambda c, cn: "grid")
    _check_order(seq, pr, lambda o: (0 * o, 0 * o), lambda c, cn: "wg")
    with pytest.raises(AssertionError):
        _check_order(seq, pr, lambda o: (0 * o, o), lambda c, cn: "none")  # same workgroup, other wave
    with pytest.raises(AssertionError):  # and same-colour conflicts
        _check_same_colour([[0, 1]], {0: {"x"}, 1: {"x"}})
