"""Writes tests/golden/rank_pairs_cfg123.npz: (features, rank) pairs of the
oracle's factorizations of the three single-system workloads (2-D Laplacian
64x64 leaf 64, slab 64x64x16 leaf 256, two-component slab 128x128x20 leaf
256; tolerance 1e-2), the training set of the rank MLP.  Calls only the
oracle and the input generators.

    python tests/golden/make_rank_pairs.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import learned  # noqa: E402
from synth import config  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rank_pairs_cfg123.npz")


def main():
    Xs, ks, lvs, srcs = [], [], [], []
    for si, name in enumerate(("laplace64", "slab64", "stokes128")):
        pr = config(name)
        t0 = time.time()
        X, k, lv = learned.rank_pairs(pr, pr.leaf, pr.tol)
        print(f"{name}: {len(k)} pairs, {time.time() - t0:.1f} s", flush=True)
        Xs.append(X)
        ks.append(k)
        lvs.append(lv)
        srcs.append(np.full(len(k), si))
    np.savez_compressed(OUT, X=np.concatenate(Xs), k=np.concatenate(ks), level=np.concatenate(lvs),
                        source=np.concatenate(srcs), names=np.array(["laplace64", "slab64", "stokes128"]))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
