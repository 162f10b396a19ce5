"""Writes dc_sweep.json: iterations of the oracle's factor with and without
deferred compression over tolerances and horizontal refinement.

The synthetic analogue of the paper's iteration tables (Numerical Results,
"Extruded partitioning" and "Deferred-compression scheme"): thin extruded
two-component slabs with the ice sheet's boundary types (Neumann top and
sides, a Robin bed that is zero under a floating shelf over half of the
domain: ``synth.slab_icesheet``), a fixed number of layers (9) and growing
horizontal size (each step doubles both horizontal sides, four times the
unknowns, as the paper's mesh refinements do), vertical/horizontal coupling
ratio 1e4 times a log-normal coefficient field, clusters of about 128
unknowns; the factor is the right preconditioner of GMRES(200) at 1e-12 (the
paper's Krylov wrapper) and also of PCG at 1e-8.  Every value comes from
``oracle/`` only.

    python tests/golden/make_dc_sweep.py [--sizes 12,24,48] [--jobs 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LAYERS = 9
RATIO = 1e4
LEAF = 128
TOLS = (1e-1, 1e-2, 1e-3, 1e-4)


def run_one(args):
    nh, tol, dc = args
    import threadpoolctl

    import oracle
    from oracle.gmres import gmres
    from synth import lognormal_field, rhs, slab_icesheet

    with threadpoolctl.threadpool_limits(1):
        pr = slab_icesheet(nh, nh, LAYERS, RATIO, lognormal_field((nh, nh, LAYERS), seed=1))
        T = oracle.build_tree(pr.grid, LEAF)
        rec = {"nh": nh, "n": pr.n, "tol": tol, "dc": dc}
        t0 = time.perf_counter()
        try:
            F = oracle.factor(pr.rowptr, pr.col, pr.val, T, tol, dc=dc)
        except oracle.NotSPDError as e:
            rec.update(breakdown=f"level {e.level} cluster {e.cluster}")
            return rec
        rec["factor_s"] = round(time.perf_counter() - t0, 2)
        rec["ranks_mean"] = [round(sum(lv.ranks) / max(1, len(lv.ranks)), 2) for lv in F.levels]
        A = pr.scipy()
        b = rhs(pr.n, 0)
        M = (lambda r: oracle.solve(F, r))
        _, it, rr, ok = gmres(lambda v: A @ v, b, M, 1e-12, restart=200, maxit=1000)
        rec.update(gmres_iters=it if ok else None, gmres_relres=rr)
        _, it, rr, ok = oracle.pcg(lambda v: A @ v, b, M, 1e-8, maxit=1000)
        rec.update(pcg_iters=it if ok else None, pcg_relres=rr)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="12,24,48,96")
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--out", default=os.path.join(HERE, "dc_sweep.json"))
    a = ap.parse_args()
    sizes = [int(s) for s in a.sizes.split(",")]
    work = [(nh, tol, dc) for nh in sizes for tol in TOLS for dc in (False, True)]
    work.sort(key=lambda w: -w[0])  # largest first
    with ProcessPoolExecutor(max_workers=a.jobs) as ex:
        recs = list(ex.map(run_one, work))
    for r in recs:
        print(r, flush=True)
    recs.sort(key=lambda r: (r["nh"], not r["dc"], -r["tol"]))
    with open(a.out, "w") as f:
        json.dump({"generator": "slab_icesheet (shelf_frac 0.5, beta 1e2)", "layers": LAYERS, "ratio": RATIO,
                   "leaf": LEAF, "field_seed": 1, "rhs_seed": 0,
                   "gmres": {"restart": 200, "rtol": 1e-12, "maxit": 1000}, "pcg_rtol": 1e-8,
                   "runs": recs}, f, indent=1)


if __name__ == "__main__":
    main()
