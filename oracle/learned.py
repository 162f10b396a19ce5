"""Learned-rank form (oracle side): sketch features, the rank MLP in fp64,
and the (features, rank) training pairs of oracle factorizations.

Test infrastructure: only the tests, the smoke check and the CPU baseline
of the benchmark use this module.

Random numbers.  The sketch matrix is drawn from Philox4x32-10 (Salmon,
Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011):
a counter-based generator, so both sides draw the same matrix from the same
counters without sharing state.  Gaussians come from the Box-Muller
transform of two 32-bit words u -> (u + 0.5) / 2^32.

Features of cluster s at the START of a level (reading of the learned-rank
form: at level start every link of s is a neighbour link, the far field of
s only appears as fill while the level is eliminated, so the values are
taken from the coupling whose Schur products form that fill, and the size of
the far field from the symbolic elimination of the level):
    B   = D_s^{-1/2} A_{s,n(s)} D_n^{-1/2}   (D = diagonals of the diagonal blocks)
    Y   = B Omega,  Omega[(y, j), c] = Gaussian(level, y, j, c), c < 8
    sig = singular values of Y (square roots of the eigenvalues of Y^T Y)
    f   = [log2(1+m), log2(1+b), log10(||B||_F), sig/||B||_F (8), e]
with m the size of s, b the summed level-start sizes of its far field w(s)
when it is processed, and e the fraction of its neighbours processed before
it.  The MLP (12 -> 64 -> 64 -> 1, ReLU, inputs standardised by stored mean
and inverse deviation) regresses the rank k that the elimination then finds.
"""
from __future__ import annotations

import numpy as np

NFEAT = 12
NHID = 64
NSKETCH = 8

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: uint array [..., 4], key: [..., 2]
    (broadcast); returns uint64 array [..., 4] of 32-bit words."""
    c = np.asarray(ctr, dtype=np.uint64) & _MASK
    k = np.asarray(key, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = k[..., 0], k[..., 1]
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(_W0)) & _MASK
            k1 = (k1 + np.uint64(_W1)) & _MASK
        p0 = np.uint64(_M0) * c0
        p1 = np.uint64(_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1)


def box_muller(u0, u1):
    """Two standard normals from two 32-bit words."""
    a = (np.asarray(u0, dtype=np.float64) + 0.5) * 2.0 ** -32
    b = (np.asarray(u1, dtype=np.float64) + 0.5) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(a))
    return r * np.cos(2.0 * np.pi * b), r * np.sin(2.0 * np.pi * b)


SKETCH_SEED = 0x5EED1811


def omega(level: int, cluster: int, m: int, seed: int = SKETCH_SEED) -> np.ndarray:
    """Rows of the sketch matrix for the m DoFs of one cluster: [m, 8].
    Counter (j, cluster, call, level), key (seed, 0); call c gives the
    Gaussians of columns 4c .. 4c+3."""
    j = np.arange(m, dtype=np.uint64)
    out = np.zeros((m, NSKETCH))
    for call in range(2):
        ctr = np.stack([j, np.full(m, cluster, np.uint64), np.full(m, call, np.uint64),
                        np.full(m, level, np.uint64)], axis=-1)
        w = philox4x32_10(ctr, np.array([seed, 0], dtype=np.uint64))
        g0, g1 = box_muller(w[:, 0], w[:, 1])
        g2, g3 = box_muller(w[:, 2], w[:, 3])
        out[:, 4 * call:4 * call + 4] = np.stack([g0, g1, g2, g3], axis=-1)
    return out


def symbolic_far_field(graph, sizes):
    """Processing order of the level ((colour, index), greedy distance-2
    colouring) and, per cluster, the summed sizes of its far field when it
    is processed and the fraction of its neighbours processed before it.
    The far field is every cluster linked to s but not a neighbour; the
    elimination of s links every two of its neighbours."""
    from .tree import d2_colouring
    M = len(sizes)
    col = d2_colouring(graph)
    order = sorted(range(M), key=lambda s: (col[s], s))
    pos = {s: i for i, s in enumerate(order)}
    nbr = [set(g) for g in graph]
    linked = [set(g) for g in graph]
    bsum = np.zeros(M)
    before = np.zeros(M)
    for s in order:
        bsum[s] = sum(sizes[q] for q in linked[s] if q not in nbr[s])
        before[s] = sum(1 for y in graph[s] if pos[y] < pos[s]) / max(1, len(graph[s]))
        for p in graph[s]:
            for q in graph[s]:
                if p != q:
                    linked[p].add(q)
    return bsum, before


def level_features(li: int, blocks: dict, sizes, graph, tol: float) -> np.ndarray:
    """Features [M, 12] of every cluster from the level-start blocks (a dict
    (p, q) -> dense block, diagonal blocks by their lower triangle).  tol is
    not a feature (the network is trained at one tolerance)."""
    M = len(sizes)
    bsum, before = symbolic_far_field(graph, sizes)
    diag = [np.diag(blocks[(p, p)]).astype(np.float64) if sizes[p] else np.zeros(0) for p in range(M)]
    isq = [1.0 / np.sqrt(d) if d.size else d for d in diag]
    om = [omega(li, p, sizes[p]) for p in range(M)]
    F = np.zeros((M, NFEAT))
    for s in range(M):
        m = sizes[s]
        Y = np.zeros((m, NSKETCH))
        fro2 = 0.0
        for y in graph[s]:
            if m == 0 or sizes[y] == 0:
                continue
            B = (isq[s][:, None] * blocks[(s, y)]) * isq[y][None, :]
            fro2 += float(np.sum(B * B))
            Y += B @ om[y]
        fro = np.sqrt(fro2)
        ev = np.linalg.eigvalsh(Y.T @ Y) if m else np.zeros(NSKETCH)
        sig = np.sqrt(np.maximum(ev[::-1], 0.0))
        F[s, 0] = np.log2(1.0 + m)
        F[s, 1] = np.log2(1.0 + bsum[s])
        F[s, 2] = np.log10(fro + 1e-300)
        F[s, 3:3 + NSKETCH] = sig / max(fro, 1e-300)
        F[s, 11] = before[s]
    return F


# ---- MLP ------------------------------------------------------------------
# Packed parameters (float32 on the device, float64 here):
#   mu[12], isd[12], W1[64][12], b1[64], W2[64][64], b2[64], w3[64], b3
_SHAPES = [("mu", (NFEAT,)), ("isd", (NFEAT,)), ("W1", (NHID, NFEAT)), ("b1", (NHID,)),
           ("W2", (NHID, NHID)), ("b2", (NHID,)), ("w3", (NHID,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in _SHAPES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shp in _SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def pack(d) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in _SHAPES])


def mlp_forward(params, X):
    """Predicted ranks [n] and the hidden activations."""
    P = unpack(params)
    Xs = (np.asarray(X, dtype=np.float64) - P["mu"]) * P["isd"]
    z1 = Xs @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["w3"] + P["b3"][0]
    return y, (Xs, z1, h1, z2, h2)


def mlp_loss_grad(params, X, t):
    """Loss 0.5*mean((y - t)^2) and its gradient by backpropagation (the
    gradients of mu and isd are zero: they are fixed by the data)."""
    P = unpack(params)
    y, (Xs, z1, h1, z2, h2) = mlp_forward(params, X)
    n = len(y)
    r = y - np.asarray(t, dtype=np.float64)
    loss = 0.5 * float(np.mean(r * r))
    dy = r / n
    g = {name: np.zeros(shp) for name, shp in _SHAPES}
    g["w3"] = h2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, P["w3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ Xs
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


# ---- training pairs ---------------------------------------------------------
def rank_pairs(problem, leaf: int, tol: float):
    """(features [N, 12], ranks [N], level [N]) over every eliminated level
    of the oracle's factorization of one problem."""
    from .hsolver import factor
    from .tree import build_tree
    feats = []

    def hook(li, blocks, sizes, graph):
        feats.append(level_features(li, blocks, sizes, graph, tol))

    T = build_tree(problem.grid, leaf)
    F = factor(problem.rowptr, problem.col, problem.val, T, tol, level_hook=hook)
    X, k, lv = [], [], []
    for li, rec in enumerate(F.levels):
        X.append(feats[li])
        k.append(np.asarray(rec.ranks, dtype=np.float64))
        lv.append(np.full(len(rec.ranks), li))
    return np.concatenate(X), np.concatenate(k), np.concatenate(lv)
