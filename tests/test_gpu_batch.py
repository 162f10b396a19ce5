"""Batching form through the C-ABI: many independent systems per launch.

Each system of a batch must get exactly the factor the single-system path
computes with one persistent launch per level (same kernels per cluster),
so schedules, ranks and M^{-1} b are compared bit for bit with it, and with
the oracle to the usual bars (schedule bit-exact, apply <= 1e-10, PCG +-1
iteration and <= 1e-8).  The replayed graphs of the refactorization and of
PCG are checked against eager runs on every replay.
"""
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle
from synth import batch_params, batch_rhs, batch_system, lognormal_field, slab_scalar

pytestmark = pytest.mark.gpu

APPLY_TOL = 1e-10


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def L():
    from paper_1811_11248_amd import lrsp
    return lrsp


def _problems():
    """Four of the smallest draws of the many-systems workload, two draws
    whose largest leaves hold 275 and 325 DoFs (157 of the 512 systems have
    leaves above 256), one system whose graph is a single cluster (dense top
    at level 0) and one with a small leaf (more levels than the others)."""
    P = batch_params()
    out = [(batch_system(i, P), 256) for i in (196, 456, 7, 22, 214, 466)]
    tiny = slab_scalar(4, 4, 8, 1e3, lognormal_field((4, 4, 8), seed=9))
    out.append((tiny, 256))
    deep = slab_scalar(12, 10, 6, 1e4, lognormal_field((10, 12, 6), seed=4))
    out.append((deep, 48))
    return out


_CACHE = {}


def _setup(torch, L):
    if "probs" not in _CACHE:
        probs = _problems()
        oracles = []
        for pr, leaf in probs:
            T = oracle.build_tree(pr.grid, leaf)
            oracles.append(oracle.factor(pr.rowptr, pr.col, pr.val, T, 1e-2))
        _CACHE["probs"] = probs
        _CACHE["oracles"] = oracles
    probs = _CACHE["probs"]
    mats = [L.DeviceMatrix.from_problem(pr) for pr, _ in probs]
    trees = [L.Tree(pr.grid, leaf) for pr, leaf in probs]
    return probs, _CACHE["oracles"], mats, trees


def _packed_rhs(probs, nrhs):
    return [batch_rhs(i, pr.n, nrhs) for i, (pr, _) in enumerate(probs)]


def test_batch_matches_single_and_oracle(torch, L):
    L.autotune_clear()
    probs, oracles, mats, trees = _setup(torch, L)
    _say(f"[batch] {len(probs)} systems, n = {[pr.n for pr, _ in probs]}")
    B = L.Batch(mats, trees, 1e-2)
    torch.cuda.synchronize()
    info = B.info()
    _say(f"  info {info}")
    assert (B.status == 0).all()
    bs = _packed_rhs(probs, 2)
    X = B.apply(B.pack(bs)).cpu().numpy()
    for i, ((pr, leaf), Fo) in enumerate(zip(probs, oracles)):
        _say(f"  system {i}: n={pr.n} leaf={leaf} oracle levels={len(Fo.levels)}")
        assert B.system_levels(i) == len(Fo.levels)
        for li, lv in enumerate(Fo.levels):
            g = B.level(i, li)
            assert g["sizes"].tolist() == list(lv.sizes), f"sizes sys {i} level {li}"
            assert g["graph"] == [list(x) for x in lv.graph], f"graph sys {i} level {li}"
            assert g["colour"].tolist() == list(lv.colour), f"colour sys {i} level {li}"
            assert g["order"].tolist() == list(lv.order), f"order sys {i} level {li}"
            assert g["ranks"].tolist() == list(lv.ranks), f"ranks sys {i} level {li}"
        assert B.level(i, len(Fo.levels))["sizes"].tolist() == list(Fo.top_sizes)
        xi = X[B.off[i]:B.off[i + 1]]
        # single-system path with one persistent launch per level: same bits
        F = L.Factor(mats[i], trees[i], 1e-2, exec_mode="level")
        for c in range(2):
            xs = L.apply(F, torch.from_numpy(bs[i][:, c].copy()).cuda()).cpu().numpy()
            assert np.array_equal(xs, xi[:, c]), f"sys {i} col {c} differs from the single path"
            xo = oracle.solve(Fo, bs[i][:, c])
            err = np.linalg.norm(xi[:, c] - xo) / np.linalg.norm(xo)
            assert err <= APPLY_TOL, f"sys {i} col {c}: {err:.3e}"


@pytest.mark.parametrize("mode", ["split", "colour", "level"])
def test_batch_forced_schedules(torch, L, mode):
    """Every level forced to one schedule (several workgroups per cluster,
    one launch per colour, one persistent launch per level): schedules and
    ranks equal the oracle's, M^{-1} b matches it to 1e-10 (2-norm and
    element-wise), including the clusters of more than 256 DoFs."""
    L.autotune_clear()
    probs, oracles, mats, trees = _setup(torch, L)
    _say(f"[batch forced {mode}] {len(probs)} systems, largest leaves "
         f"{[max(len(d) for d in oracle.build_tree(pr.grid, leaf).leaf_dofs) for pr, leaf in probs]}")
    B = L.Batch(mats, trees, 1e-2, exec_mode=mode)
    torch.cuda.synchronize()
    assert (B.status == 0).all()
    bs = _packed_rhs(probs, 2)
    X = B.apply(B.pack(bs)).cpu().numpy()
    for i, ((pr, leaf), Fo) in enumerate(zip(probs, oracles)):
        assert B.system_levels(i) == len(Fo.levels)
        for li, lv in enumerate(Fo.levels):
            g = B.level(i, li)
            assert g["order"].tolist() == list(lv.order), f"order sys {i} level {li}"
            assert g["ranks"].tolist() == list(lv.ranks), f"ranks sys {i} level {li}"
        xi = X[B.off[i]:B.off[i + 1]]
        F = L.Factor(mats[i], trees[i], 1e-2, exec_mode=mode)
        for c in range(2):
            xo = oracle.solve(Fo, bs[i][:, c])
            err = np.linalg.norm(xi[:, c] - xo) / np.linalg.norm(xo)
            erri = np.max(np.abs(xi[:, c] - xo)) / np.max(np.abs(xo))
            xs = L.apply(F, torch.from_numpy(bs[i][:, c].copy()).cuda()).cpu().numpy()
            _say(f"  sys {i} col {c}: n={pr.n} err {err:.2e} (element-wise {erri:.2e}), "
                 f"same bits as the single-system {mode} schedule: {np.array_equal(xs, xi[:, c])}")
            assert err <= APPLY_TOL and erri <= APPLY_TOL, f"sys {i} col {c}"


def test_batch_top_dense_threshold(torch, L):
    """The size threshold of the dense top in the batch: every system stops
    where its own factorization with the same option stops (same bits as
    the single-system path, one persistent launch per level), and matches
    the oracle with that threshold."""
    L.autotune_clear()
    probs, oracles, mats, trees = _setup(torch, L)
    thr = 400
    B = L.Batch(mats, trees, 1e-2, top_dense=thr)
    bs = _packed_rhs(probs, 1)
    X = B.apply(B.pack(bs)).cpu().numpy()
    for i, (pr, leaf) in enumerate(probs):
        Fo = oracle.factor(pr.rowptr, pr.col, pr.val, oracle.build_tree(pr.grid, leaf), 1e-2, top_dense=thr)
        assert B.system_levels(i) == len(Fo.levels)
        assert B.level(i, len(Fo.levels))["sizes"].tolist() == list(Fo.top_sizes)
        xi = X[B.off[i]:B.off[i + 1], 0]
        F = L.Factor(mats[i], trees[i], 1e-2, exec_mode="level", top_dense=thr)
        xs = L.apply(F, torch.from_numpy(bs[i][:, 0].copy()).cuda()).cpu().numpy()
        assert np.array_equal(xs, xi), f"sys {i}"
        xo = oracle.solve(Fo, bs[i][:, 0])
        assert np.linalg.norm(xi - xo) <= APPLY_TOL * np.linalg.norm(xo)


def test_batch_pcg_four_rhs(torch, L):
    L.autotune_clear()
    probs, oracles, mats, trees = _setup(torch, L)
    B = L.Batch(mats, trees, 1e-2)
    bs = _packed_rhs(probs, 4)
    Bt = B.pack(bs)
    _say("[batch pcg] 4 rhs")
    X, it, rr = B.pcg(Bt)
    torch.cuda.synchronize()
    _say(f"  iters {it.tolist()} graph_pcg={B.info()['graph_pcg']}")
    assert (rr <= 1e-8).all(), rr
    Xn = X.cpu().numpy()
    for i, ((pr, _), Fo) in enumerate(zip(probs, oracles)):
        A = pr.scipy()
        for c in range(4):
            _, ito, rro, ok = oracle.pcg(lambda v: A @ v, bs[i][:, c], lambda r: oracle.solve(Fo, r), 1e-8)
            assert ok
            assert abs(int(it[c, i]) - ito) <= 1, f"sys {i} col {c}: {it[c, i]} vs oracle {ito}"
            xi = Xn[B.off[i]:B.off[i + 1], c]
            res = np.linalg.norm(bs[i][:, c] - A @ xi) / np.linalg.norm(bs[i][:, c])
            assert res <= 1e-8


def test_pcg_graph_replays_match_eager(torch, L):
    L.autotune_clear()
    probs, oracles, mats, trees = _setup(torch, L)
    B = L.Batch(mats, trees, 1e-2)
    Bt = B.pack(_packed_rhs(probs, 4))
    # eager reference: with timing on, PCG runs without graphs
    L.timing_enable(True)
    Xe, ite, _ = B.pcg(Bt)
    Xe = Xe.clone()
    L.timing_enable(False)
    assert B.info()["graph_pcg"] == 0
    for rep in range(3):
        _say(f"[pcg graph replay {rep}]")
        Xg, itg, rrg = B.pcg(Bt)
        torch.cuda.synchronize()
        assert B.info()["graph_pcg"] == 1
        assert B.info()["graph_timeouts"] == 0
        assert np.array_equal(itg, ite)
        assert torch.equal(Xg, Xe), f"replay {rep} differs from the eager run"
        # eager work of the program between replays
        _ = B.apply(Bt)
        torch.cuda.synchronize()


def test_refactor_replays_graph(torch, L):
    L.autotune_clear()
    probs, oracles, mats, trees = _setup(torch, L)
    B = L.Batch(mats, trees, 1e-2)
    Bt = B.pack(_packed_rhs(probs, 1))
    x0 = B.apply(Bt).clone()
    for rep in range(3):
        _say(f"[refactor same values {rep}]")
        B.refactor()
        torch.cuda.synchronize()
        inf = B.info()
        assert inf["graph_factor"] == 1 and inf["refactor_fallbacks"] == 0 and inf["graph_timeouts"] == 0
        assert torch.equal(B.apply(Bt), x0), f"replay {rep} differs"
    # new value arrays, perturbed by a relative 2^-40: no rank decision is
    # that close, so the graph stays valid, and the result equals a fresh
    # factorization of the perturbed systems bit for bit
    mats2 = [L.DeviceMatrix(A.h_rowptr, A.h_col, (1.0 + 2.0 ** -40) * A.val.cpu().numpy()) for A in mats]
    _say("[refactor perturbed values]")
    B.refactor(mats2)
    assert B.info()["refactor_fallbacks"] == 0 and B.info()["graph_factor"] == 1
    fresh = L.Batch(mats2, trees, 1e-2)
    assert torch.equal(B.apply(Bt), fresh.apply(Bt))
    # other coefficients: ranks change, the batch is planned again
    probs3 = []
    for i, (pr, _) in enumerate(probs):
        nx, ny, nz, _c = pr.grid
        probs3.append(slab_scalar(nx, ny, nz, 1e2, lognormal_field((ny, nx, nz), seed=77 + i)))
    mats3 = [L.DeviceMatrix.from_problem(p) for p in probs3]
    _say("[refactor new coefficients]")
    B.refactor(mats3)
    assert B.info()["refactor_fallbacks"] == 1
    fresh3 = L.Batch(mats3, trees, 1e-2)
    assert torch.equal(B.apply(Bt), fresh3.apply(Bt))
    # the planned-again batch records a new graph on its next refactorization
    B.refactor(mats3)
    assert B.info()["graph_factor"] == 1
    assert torch.equal(B.apply(Bt), fresh3.apply(Bt))


def test_autotune_records_and_keeps_parity(torch, L):
    L.autotune_clear()
    probs, oracles, mats, trees = _setup(torch, L)
    _say("[autotune]")
    B = L.Batch(mats, trees, 1e-2, autotune=True)
    inf = B.info()
    _say(f"  sched {inf['sched']} caps {inf['grid_cap']}")
    assert inf["tuned_levels"] == inf["nlevels"] and L.autotune_entries() >= 1
    bs = _packed_rhs(probs, 1)
    X = B.apply(B.pack(bs)).cpu().numpy()
    for i, Fo in enumerate(oracles):
        xo = oracle.solve(Fo, bs[i][:, 0])
        xi = X[B.off[i]:B.off[i + 1], 0]
        assert np.linalg.norm(xi - xo) <= APPLY_TOL * np.linalg.norm(xo)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        L.autotune_save(path)
        n = L.autotune_entries()
        L.autotune_clear()
        L.autotune_load(path)
        assert L.autotune_entries() == n
    B2 = L.Batch(mats, trees, 1e-2)  # uses the table
    assert B2.info()["sched"][:inf["nlevels"]] == inf["sched"][:inf["nlevels"]]
    L.autotune_clear()


def test_autotune_tile_shapes_keep_bits(torch, L):
    """The tuner's tile choice for the split schedule (16 or 32 columns per
    workgroup in the scaling step) changes the launch, not the arithmetic:
    with every level forced to the split schedule through the table, both
    tiles give the same bits, and the batch reports the tile it used."""
    import re
    L.autotune_clear()
    probs, oracles, mats, trees = _setup(torch, L)
    B = L.Batch(mats, trees, 1e-2, autotune=True)
    inf = B.info()
    _say(f"[autotune tiles] sched {inf['sched']} tiles {inf['tile']}")
    Bt = B.pack(_packed_rhs(probs, 1))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        L.autotune_save(path)
        text = open(path).read()
        assert '"tile"' in text
        X = {}
        for tile in (1, 0):
            t2 = re.sub(r'"sched": \d+', '"sched": 2', text)
            t2 = re.sub(r'"tile": \d+', f'"tile": {tile}', t2)
            with open(path, "w") as f:
                f.write(t2)
            L.autotune_clear()
            L.autotune_load(path)
            Bf = L.Batch(mats, trees, 1e-2)  # schedules and tiles from the table
            fi = Bf.info()
            assert all(sc == "split" for sc in fi["sched"][:fi["nlevels"]])
            assert all(t == (16 if tile else 32) for t in fi["tile"][:fi["nlevels"]])
            X[tile] = Bf.apply(Bt).clone()
    L.autotune_clear()
    assert torch.equal(X[0], X[1])
    Xn = X[1].cpu().numpy()
    for i, Fo in enumerate(oracles):
        xo = oracle.solve(Fo, _packed_rhs(probs, 1)[i][:, 0])
        xi = Xn[B.off[i]:B.off[i + 1]].ravel()
        assert np.linalg.norm(xi - xo) <= APPLY_TOL * np.linalg.norm(xo)


def test_not_spd_system_is_reported(torch, L):
    L.autotune_clear()
    probs, oracles, mats, trees = _setup(torch, L)
    bad = L.DeviceMatrix(mats[1].h_rowptr, mats[1].h_col, -mats[1].val.cpu().numpy())
    mats_b = [mats[0], bad, mats[2]]
    _say("[batch with one indefinite system]")
    B = L.Batch(mats_b, trees[:3], 1e-2, raise_not_spd=False)
    assert B.status.tolist() == [0, L.ERR_NOT_SPD, 0]
    bs = [batch_rhs(i, m.n, 1) for i, m in enumerate(mats_b)]
    X = B.apply(B.pack(bs)).cpu().numpy()
    # the other systems are untouched: same bits as a batch without the bad one
    G = L.Batch([mats[0], mats[2]], [trees[0], trees[2]], 1e-2)
    Y = G.apply(G.pack([bs[0], bs[2]])).cpu().numpy()
    assert np.array_equal(X[B.off[0]:B.off[1]], Y[G.off[0]:G.off[1]])
    assert np.array_equal(X[B.off[2]:B.off[3]], Y[G.off[1]:G.off[2]])
