"""Parity of the elimination WITHOUT deferred compression (scheme 1) with the
oracle's ``factor(dc=False)``, through the C-ABI.

The scheme the paper compares against (section Deferred-compression Scheme,
Eqs. offdiag and sc_old): the unscaled far-field block is compressed, the
cluster rotated and its fine part eliminated; the coarse unknowns keep a
Schur-complement diagonal block instead of the identity.  Bars as for the
scaled form: schedule and ranks equal the oracle's bit for bit, M^{-1} b
matches the oracle's solve to relative 1e-10 in fp64 (2-norm and element by
element), PCG iteration counts within one of the oracle's; at tol = 0 the
factor is exact.  The sweep over tolerances on the ice-sheet analogue is
compared with the stored oracle iteration counts (``golden/dc_sweep.json``,
written by ``golden/make_dc_sweep.py`` from the oracle only): GMRES(200) at
1e-12 within one iteration, with and without deferred compression.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from synth import laplace2d, lognormal_field, rhs, slab_icesheet, slab_scalar, slab_vector

pytestmark = pytest.mark.gpu

APPLY_TOL = 1e-10
HERE = os.path.dirname(os.path.abspath(__file__))


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


CASES = {
    "laplace16": (lambda: laplace2d(16), 16, 1e-2),
    "slab_ragged": (lambda: slab_scalar(13, 11, 5, 1e3, lognormal_field((11, 13, 5), seed=2)), 40, 1e-2),
    "vector_ragged": (lambda: slab_vector(10, 9, 4, 1e2), 48, 1e-2),
    "slab_aniso": (lambda: slab_scalar(24, 20, 8, 1e4, lognormal_field((20, 24, 8), seed=5)), 64, 1e-3),
    "slab_tol0": (lambda: slab_scalar(8, 8, 4, 1e3, lognormal_field((8, 8, 4), seed=3)), 16, 0.0),
    "strip4": (lambda: laplace2d(32, 2), 16, 0.5),
    "single_cluster": (lambda: laplace2d(6), 64, 1e-2),
    # clusters of 96..160 DoFs: the column operations from global memory
    "slab_split": (lambda: slab_scalar(24, 20, 8, 1e4, lognormal_field((20, 24, 8), seed=7)), 128, 1e-2),
    # clusters of 216..384 DoFs: the sweeps of large clusters (split units)
    "slab_large": (lambda: slab_scalar(13, 13, 24, 1e4, lognormal_field((13, 13, 24), seed=8)), 256, 1e-2),
    # the ice-sheet analogue (floating shelf, Robin bed) at two tolerances
    "icesheet_1e-1": (lambda: slab_icesheet(12, 12, 9, 1e4, lognormal_field((12, 12, 9), seed=1)), 128, 1e-1),
    "icesheet_1e-3": (lambda: slab_icesheet(12, 12, 9, 1e4, lognormal_field((12, 12, 9), seed=1)), 128, 1e-3),
}
MODES = ["colour", "level"]

_ORACLE = {}


def _oracle(name):
    if name not in _ORACLE:
        mk, leaf, tol = CASES[name]
        pr = mk()
        T = oracle.build_tree(pr.grid, leaf)
        _ORACLE[name] = (pr, oracle.factor(pr.rowptr, pr.col, pr.val, T, tol, dc=False))
    return _ORACLE[name]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", list(CASES))
def test_nodc_schedule_and_apply(torch, L, name, mode):
    mk, leaf, tol = CASES[name]
    pr, Fo = _oracle(name)
    _say(f"[nodc case {name} / {mode}] n={pr.n} leaf={leaf} tol={tol}")
    A = L.DeviceMatrix.from_problem(pr)
    F = L.Factor(A, L.Tree(pr.grid, leaf), tol, exec_mode=mode, dc=False)
    torch.cuda.synchronize()
    exact = tol == 0.0
    if not exact:
        assert F.info()["nlevels"] == len(Fo.levels)
    for li, lv in enumerate(Fo.levels[:1] if exact else Fo.levels):
        g = F.level(li)
        assert g["sizes"].tolist() == list(lv.sizes), f"sizes level {li}"
        assert g["order"].tolist() == list(lv.order), f"order level {li}"
        if not exact:
            assert g["ranks"].tolist() == list(lv.ranks), f"ranks level {li}"
    if not exact:
        assert F.level(len(Fo.levels))["sizes"].tolist() == list(Fo.top_sizes)
    for seed in (0, 1):
        b = rhs(pr.n, seed)
        xo = oracle.solve(Fo, b)
        x = L.apply(F, torch.from_numpy(b).cuda()).cpu().numpy()
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        erri = np.max(np.abs(x - xo)) / np.max(np.abs(xo))
        _say(f"  apply rel err {err:.3e} (element-wise {erri:.3e})")
        assert err <= APPLY_TOL
        assert erri <= APPLY_TOL
    if exact:
        xe = np.linalg.solve(pr.scipy().toarray(), b)
        assert np.linalg.norm(x - xe) <= 1e-10 * np.linalg.norm(xe)


@pytest.mark.parametrize("name", ["slab_aniso", "slab_split", "icesheet_1e-1"])
def test_nodc_pcg_iterations(torch, L, name):
    mk, leaf, tol = CASES[name]
    pr, Fo = _oracle(name)
    _say(f"[nodc pcg {name}] n={pr.n}")
    As = pr.scipy()
    b = rhs(pr.n, 0)
    _, ito, _, ok = oracle.pcg(lambda v: As @ v, b, lambda r: oracle.solve(Fo, r), 1e-8)
    assert ok
    A = L.DeviceMatrix.from_problem(pr)
    F = L.Factor(A, L.Tree(pr.grid, leaf), tol, dc=False)
    x, it, rr = L.pcg(A, F, torch.from_numpy(b).cuda(), rtol=1e-8)
    _say(f"  iterations {int(it[0])} (oracle {ito})")
    assert abs(int(it[0]) - ito) <= 1
    r = b - As @ x.cpu().numpy()
    assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(b)


def test_nodc_tree_and_scheme_options(torch, L):
    # scheme 1 with the learned rank form, and the batching form, are refused
    pr = laplace2d(16)
    A = L.DeviceMatrix.from_problem(pr)
    with pytest.raises(L.LrspError):
        L.Factor(A, L.Tree(pr.grid, 16), 1e-2, dc=False, mlp=np.zeros(L.mlp_nparams(), np.float32))
    # the scaled form and scheme 1 agree where no far field exists (a strip
    # of four clusters: every step is plain block Cholesky)
    pr = laplace2d(32, 2)
    A = L.DeviceMatrix.from_problem(pr)
    b = torch.from_numpy(rhs(pr.n, 3)).cuda()
    x1 = L.apply(L.Factor(A, L.Tree(pr.grid, 16), 0.5, dc=False), b).cpu().numpy()
    x0 = L.apply(L.Factor(A, L.Tree(pr.grid, 16), 0.5), b).cpu().numpy()
    assert np.linalg.norm(x1 - x0) <= 1e-12 * np.linalg.norm(x0)


def _golden():
    with open(os.path.join(HERE, "golden", "dc_sweep.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("nh", [12, 24])
def test_dc_sweep_matches_stored_oracle_counts(torch, L, nh):
    g = _golden()
    runs = [r for r in g["runs"] if r["nh"] == nh]
    assert runs
    pr = slab_icesheet(nh, nh, g["layers"], g["ratio"], lognormal_field((nh, nh, g["layers"]), seed=g["field_seed"]))
    A = L.DeviceMatrix.from_problem(pr)
    T = L.Tree(pr.grid, g["leaf"])
    b = torch.from_numpy(rhs(pr.n, g["rhs_seed"])).cuda()
    gm = g["gmres"]
    for r in runs:
        F = L.Factor(A, T, r["tol"], dc=r["dc"])
        _, it, rr = L.gmres(A, F, b, rtol=gm["rtol"], restart=gm["restart"], maxit=gm["maxit"])
        _say(f"  nh {nh} tol {r['tol']} dc {r['dc']}: GMRES {int(it[0])} (oracle {r['gmres_iters']})")
        assert abs(int(it[0]) - r["gmres_iters"]) <= 1
        _, itp, _ = L.pcg(A, F, b, rtol=g["pcg_rtol"])
        assert abs(int(itp[0]) - r["pcg_iters"]) <= 1
