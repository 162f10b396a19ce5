"""Deferred-compression hierarchical factorization and solve (oracle).

Follows the paper's section "Improved LoRaSp Solver":

* one cluster step is the scaled low-rank elimination ``W_s = P_s G_s E_s S_s``
  (Eqs. scaling, sparse, elim, perm): Cholesky ``A_ss = G G^T``; scale the
  block row by ``G^{-1}``; compress the scaled far-field block
  ``G^{-1} A_sw = U_hat V_hat^T`` (Eq. offdiag_new); rotate the cluster by
  ``U_hat^T`` so that its fine part ``U_hat_2^T`` carries no far-field
  coupling; eliminate the fine part, which updates the near field
  ``X_nn = A_nn - F^T F`` with ``F = U_hat_2^T G^{-1} A_sn``; keep the ``k``
  coarse DoFs, whose row becomes ``[I | U_hat_1^T G^{-1} A_sn | V_hat_1^T]``;
* Algorithm 1 applies that step to every cluster of a level, then recurses on
  the coarse DoFs (parent = [left child's coarse DoFs, right child's]);
* Algorithm 2 is the forward (``y <- W_i y``) and backward (``x <- W_i^T x``)
  substitution.

Readings of points the paper leaves open (shared with the HIP path):

* neighbours ``n(s)`` are the clusters linked to ``s`` in the matrix at the
  START of the level; the far field ``w(s)`` is every other cluster linked to
  ``s`` when ``s`` is processed (fill from earlier steps of the level); a
  link is structural, so a zero-size or zero-valued block still counts;
* clusters are processed in (colour, index) order, colours from a greedy
  distance-2 colouring of the level graph in index order;
* recursion stops at the first level whose graph is complete or which has
  one cluster: plain Cholesky of all remaining DoFs in cluster order;
* diagonal blocks are represented by their lower triangle;
* the Schur update may round ``F`` to fp32 or bf16 with fp32 accumulation
  (``gemm_prec``), the rest stays fp64.

Data layout: a dict of dense blocks keyed by ordered cluster pairs, both
halves kept as exact transposes of each other.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from .cpqr import apply_q, apply_qt, cpqr
from .tree import ClusterTree, d2_colouring, level0_graph


class NotSPDError(RuntimeError):
    def __init__(self, level, cluster, msg="diagonal block not positive definite"):
        super().__init__(f"{msg} (level {level}, cluster {cluster})")
        self.level = level
        self.cluster = cluster


@dataclasses.dataclass
class SLRE:
    """Result of one scaled low-rank elimination on a block row."""
    G: np.ndarray  # m x m lower Cholesky factor of A_ss
    V: np.ndarray  # m x k Householder vectors of U_hat
    tau: np.ndarray  # k
    k: int
    C: np.ndarray  # U_hat^T G^{-1} A_sn  (m x a); rows k: are F
    Vt: np.ndarray  # V_hat_1^T in original column order (k x b)
    R: np.ndarray  # k x b pivoted R
    perm: np.ndarray  # pivot order of the columns of the w block
    margin: float = float("inf")  # distance of the rank decision from the threshold


def chol_lower(A: np.ndarray, level=-1, cluster=-1) -> np.ndarray:
    m = A.shape[0]
    if m == 0:
        return np.zeros((0, 0))
    S = np.tril(A) + np.tril(A, -1).T
    try:
        return np.linalg.cholesky(S)
    except np.linalg.LinAlgError as e:
        raise NotSPDError(level, cluster) from e


def _lsolve(G, X):
    if G.shape[0] == 0 or X.size == 0:
        return np.array(X, dtype=np.float64, copy=True)
    return scipy.linalg.solve_triangular(G, X, lower=True, check_finite=False)


def _ltsolve(G, X):
    if G.shape[0] == 0 or X.size == 0:
        return np.array(X, dtype=np.float64, copy=True)
    return scipy.linalg.solve_triangular(G, X, lower=True, trans="T", check_finite=False)


def scaled_lowrank_elimination(Ass, Asn, Asw, tol, tol_mode="relative", level=-1, cluster=-1) -> SLRE:
    """One step ``W_s`` on the block row ``[A_ss | A_sn | A_sw]``."""
    G = chol_lower(Ass, level, cluster)  # S_s, Eq. scaling
    Bn = _lsolve(G, Asn)
    Bw = _lsolve(G, Asw)
    m, b = Bw.shape
    margin = float("inf")
    if b == 0 or m == 0:
        k, V, tau, R, perm = 0, np.zeros((m, 0)), np.zeros(0), np.zeros((0, b)), np.arange(b)
    else:
        info = {}
        k, V, tau, R, perm = cpqr(Bw, tol, tol_mode, info)  # Eq. offdiag_new
        margin = decision_margin(info, tol, tol_mode)
    C = apply_qt(V, tau, Bn) if k > 0 else np.array(Bn, copy=True)  # E_s, Eq. sparse
    Vt = np.zeros((k, b))
    Vt[:, perm] = R
    return SLRE(G, V, tau, k, C, Vt, R, perm, margin)


def decision_margin(info: dict, tol: float, tol_mode: str) -> float:
    """Relative distance of the pivot norms that decided a rank from the
    threshold (the kept pivot just above it, the stopping pivot at or below
    it): a perturbation of the block smaller than this cannot change the
    rank.  Infinite when no pivot was compared with a positive threshold."""
    thr = tol * info["r00"] if tol_mode == "relative" else tol
    if not thr > 0.0:
        return float("inf")
    out = float("inf")
    for key in ("last", "stop"):
        v = info.get(key)
        if v is not None and v > 0.0:
            out = min(out, abs(v - thr) / thr)
    return out


@dataclasses.dataclass
class NoDCStep:
    """Result of one elimination step without deferred compression."""
    V: np.ndarray  # m x k Householder vectors of U (from the unscaled A_sw)
    tau: np.ndarray  # k
    k: int
    Gf: np.ndarray  # (m-k) x (m-k) lower Cholesky factor of U_2^T A_ss U_2
    Fc: np.ndarray  # Gf^{-1} U_2^T A_ss U_1  ((m-k) x k)
    Fn: np.ndarray  # Gf^{-1} U_2^T A_sn      ((m-k) x a)
    Dc: np.ndarray  # coarse diagonal block U_1^T A_ss U_1 - Fc^T Fc (k x k)
    Ccn: np.ndarray  # coarse-near coupling U_1^T A_sn - Fc^T Fn (k x a)
    Vt: np.ndarray  # V_1^T in original column order (k x b)
    R: np.ndarray
    perm: np.ndarray
    margin: float = float("inf")


def lowrank_elimination_nodc(Ass, Asn, Asw, tol, tol_mode="relative", level=-1, cluster=-1) -> NoDCStep:
    """One step of the scheme WITHOUT deferred compression (section
    Deferred-compression Scheme, Eqs. offdiag and sc_old) on the block row
    ``[A_ss | A_sn | A_sw]``: the unscaled far-field block is compressed,
    ``A_sw = U_1 V_1^T + U_2 V_2^T`` (the same column-pivoted QR and rank rule
    as the scaled form), ``U_2 V_2^T`` is dropped, the cluster is rotated by
    ``U^T`` and its fine part (the ``U_2`` directions, which no longer couple
    to the far field) is eliminated by Cholesky.  The ``k`` coarse DoFs keep
    the Schur complement of that elimination: diagonal ``Dc``, near-field
    coupling ``Ccn`` and far-field coupling ``V_1^T``; eliminating them too
    gives the approximate Schur complement ``S_A~`` of Eq. sc_old."""
    m, b = Asw.shape
    S = np.tril(Ass) + np.tril(Ass, -1).T
    margin = float("inf")
    if b == 0 or m == 0:
        k, V, tau, R, perm = 0, np.zeros((m, 0)), np.zeros(0), np.zeros((0, b)), np.arange(b)
    else:
        info = {}
        k, V, tau, R, perm = cpqr(Asw, tol, tol_mode, info)  # Eq. offdiag
        margin = decision_margin(info, tol, tol_mode)
    if k > 0:
        Bss = apply_qt(V, tau, apply_qt(V, tau, S).T)  # U^T A_ss U (A_ss symmetric)
        Bsn = apply_qt(V, tau, Asn)
    else:
        Bss, Bsn = S, np.array(Asn, dtype=np.float64, copy=True)
    Gf = chol_lower(Bss[k:, k:], level, cluster)
    Fc = _lsolve(Gf, Bss[k:, :k])
    Fn = _lsolve(Gf, Bsn[k:, :])
    Dc = Bss[:k, :k] - Fc.T @ Fc
    Dc = 0.5 * (Dc + Dc.T)
    Ccn = Bsn[:k, :] - Fc.T @ Fn
    Vt = np.zeros((k, b))
    Vt[:, perm] = R
    return NoDCStep(V, tau, k, Gf, Fc, Fn, Dc, Ccn, Vt, R, perm, margin)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) and return as float32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def schur_product(Fp: np.ndarray, Fq: np.ndarray, prec: str) -> np.ndarray:
    """``Fp^T Fq`` in the requested precision, returned as float64."""
    if prec == "f64":
        return Fp.T @ Fq
    if prec == "f32":
        a, b = Fp.astype(np.float32), Fq.astype(np.float32)
    elif prec == "bf16":
        a, b = round_bf16(Fp), round_bf16(Fq)
    else:
        raise ValueError(prec)
    return (a.T @ b).astype(np.float64)


@dataclasses.dataclass
class ClusterRecord:
    s: int
    m: int
    k: int
    a: int
    b: int
    G: np.ndarray
    V: np.ndarray
    tau: np.ndarray
    F: np.ndarray  # (m-k) x a
    nlist: list  # [(q, active width of q when s was processed)]
    wlist: list
    margin: float = float("inf")  # relative distance of the rank decision from the threshold
    Fc: np.ndarray | None = None  # without deferred compression: Gf^{-1} U_2^T A_ss U_1 (G is then Gf)


@dataclasses.dataclass
class LevelRecord:
    sizes: list
    graph: list
    colour: list
    order: list
    ranks: list
    recs: list
    min_eig: float | None = None


@dataclasses.dataclass
class Factor:
    tree: ClusterTree
    tol: float
    tol_mode: str
    gemm_prec: str
    levels: list
    top_sizes: list
    top_graph: list
    top_L: np.ndarray
    flops: dict
    corollary_min: float | None = None
    dc: bool = True


def _dense_active(blocks, sizes):
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    D = np.zeros((off[-1], off[-1]))
    for (p, q), B in blocks.items():
        D[off[p]:off[p + 1], off[q]:off[q + 1]] = B
    for p in range(len(sizes)):
        blk = D[off[p]:off[p + 1], off[p]:off[p + 1]]
        D[off[p]:off[p + 1], off[p]:off[p + 1]] = np.tril(blk) + np.tril(blk, -1).T
    return D


def _level0_blocks(tree: ClusterTree, rowptr, col, val):
    n = len(rowptr) - 1
    A = sp.csr_matrix((val, col, rowptr), shape=(n, n))
    perm = tree.perm()
    Ap = A[perm][:, perm].tocsr()
    sizes = [len(d) for d in tree.leaf_dofs]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    graph = level0_graph(tree, rowptr, col)
    blocks = {}
    for p in range(len(sizes)):
        rows = Ap[off[p]:off[p + 1]]
        blocks[(p, p)] = rows[:, off[p]:off[p + 1]].toarray()
        for q in graph[p]:
            blocks[(p, q)] = rows[:, off[q]:off[q + 1]].toarray()
    return blocks, sizes, graph


def _eliminate_level(li, blocks, sizes, graph, tol, tol_mode, prec, flops, checks, cor, dc=True):
    M = len(sizes)
    colour = d2_colouring(graph)
    order = sorted(range(M), key=lambda s: (colour[s], s))
    nbr = [set(g) for g in graph]
    linked = [set() for _ in range(M)]
    for (p, q) in blocks:
        if p != q:
            linked[p].add(q)
    cur = list(sizes)
    ranks = [0] * M
    recs = []
    for s in order:
        n = sorted(graph[s])
        w = sorted(q for q in linked[s] if q not in nbr[s])
        m = cur[s]
        nw = [cur[q] for q in n]
        ww = [cur[q] for q in w]
        Asn = np.hstack([blocks[(s, q)] for q in n]) if n else np.zeros((m, 0))
        Asw = np.hstack([blocks[(s, q)] for q in w]) if w else np.zeros((m, 0))
        if checks and w:
            # Corollary: the ww block of the DC Schur complement is SPD
            wo = np.concatenate([[0], np.cumsum(ww)]).astype(int)
            Aww = np.zeros((wo[-1], wo[-1]))
            for i, p in enumerate(w):
                for j, q in enumerate(w):
                    if (p, q) in blocks:
                        Aww[wo[i]:wo[i + 1], wo[j]:wo[j + 1]] = blocks[(p, q)]
            Aww = np.tril(Aww) + np.tril(Aww, -1).T
        if dc:
            st = scaled_lowrank_elimination(blocks[(s, s)], Asn, Asw, tol, tol_mode, li, s)
        else:
            st = lowrank_elimination_nodc(blocks[(s, s)], Asn, Asw, tol, tol_mode, li, s)
        k = st.k
        a, b = Asn.shape[1], Asw.shape[1]
        if checks and dc and w and Aww.size:
            ev = float(np.linalg.eigvalsh(Aww - st.Vt.T @ st.Vt).min())
            cor[0] = ev if cor[0] is None else min(cor[0], ev)
        flops["potrf"] += m ** 3 / 3.0
        flops["trsm"] += m * m * (a + b)
        flops["cpqr"] += sum(4.0 * (m - j) * (b - j) for j in range(k))
        flops["applyq"] += sum(4.0 * (m - j) * a for j in range(k))
        flops["schur"] += a * (a + 1.0) * (m - k)
        if dc:
            F, Cc, Dk, G = st.C[k:, :], st.C[:k, :], np.eye(k), st.G
        else:
            # the fine elimination also costs a rotation of the diagonal block
            # and the coarse block updates (not in the scaled form's count)
            F, Cc, Dk, G = st.Fn, st.Ccn, st.Dc, st.Gf
        no = np.concatenate([[0], np.cumsum(nw)]).astype(int)
        # Schur update of the near field, X_nn = A_nn - F^T F (Eq. elim)
        for i, p in enumerate(n):
            Fp = F[:, no[i]:no[i + 1]]
            for j in range(i, len(n)):
                q = n[j]
                Fq = F[:, no[j]:no[j + 1]]
                upd = schur_product(Fp, Fq, prec)
                if (p, q) not in blocks:
                    blocks[(p, q)] = np.zeros((cur[p], cur[q]))
                    linked[p].add(q)
                    linked[q].add(p)
                blocks[(p, q)] = blocks[(p, q)] - upd
                if p != q:
                    blocks[(q, p)] = blocks[(p, q)].T.copy()
        # coarse row of s: [I_k | U1^T G^-1 A_sn | V1^T] (without deferred
        # compression: [Dc | Ccn | V1^T]), then P_s moves it on
        blocks[(s, s)] = Dk
        for i, q in enumerate(n):
            blocks[(s, q)] = Cc[:, no[i]:no[i + 1]].copy()
            blocks[(q, s)] = blocks[(s, q)].T.copy()
        wo = np.concatenate([[0], np.cumsum(ww)]).astype(int)
        for i, q in enumerate(w):
            blocks[(s, q)] = st.Vt[:, wo[i]:wo[i + 1]].copy()
            blocks[(q, s)] = blocks[(s, q)].T.copy()
        cur[s] = k
        ranks[s] = k
        recs.append(ClusterRecord(s, m, k, a, b, G, st.V, st.tau, F.copy(),
                                  list(zip(n, nw)), list(zip(w, ww)), st.margin,
                                  None if dc else st.Fc.copy()))
    rec = LevelRecord(list(sizes), [list(g) for g in graph], colour, order, ranks, recs)
    if checks:
        D = _dense_active({key: B for key, B in blocks.items()}, cur)
        rec.min_eig = float(np.linalg.eigvalsh(D).min()) if D.size else None
    return rec, cur


def _coarsen(blocks, cur, M):
    P = M // 2
    sizes = [cur[2 * c] + cur[2 * c + 1] for c in range(P)]
    pairs = {(p // 2, q // 2) for (p, q) in blocks}
    nb = {}
    for (Pp, Qq) in pairs:
        B = np.zeros((sizes[Pp], sizes[Qq]))
        ro = [0, cur[2 * Pp], sizes[Pp]]
        co = [0, cur[2 * Qq], sizes[Qq]]
        for a in range(2):
            for b in range(2):
                key = (2 * Pp + a, 2 * Qq + b)
                if key in blocks:
                    B[ro[a]:ro[a + 1], co[b]:co[b + 1]] = blocks[key]
        nb[(Pp, Qq)] = B
    graph = [set() for _ in range(P)]
    for (Pp, Qq) in nb:
        if Pp != Qq:
            graph[Pp].add(Qq)
    return nb, sizes, [sorted(g) for g in graph]


def factor(rowptr, col, val, tree: ClusterTree, tol: float, tol_mode: str = "relative",
           gemm_prec: str = "f64", checks: bool = False, level_hook=None, dc: bool = True,
           top_dense: int = 0) -> Factor:
    """Algorithm 1 over the cluster tree; returns the factor of ``A``.

    The recursion stops at the first level whose cluster graph is complete or
    has one cluster, and, with ``top_dense`` > 0, also at the first level with
    at most ``top_dense`` unknowns ("small enough" to factor directly); the
    rest is one dense Cholesky in cluster order.  dc=False replaces every
    scaled low-rank elimination by the step without deferred compression
    (``lowrank_elimination_nodc``), the scheme the paper compares against.
    level_hook(level, blocks, sizes, graph), if given, sees the matrix at the
    start of every eliminated level (read only)."""
    blocks, sizes, graph = _level0_blocks(tree, rowptr, col, val)
    flops = dict(potrf=0.0, trsm=0.0, cpqr=0.0, applyq=0.0, schur=0.0, top=0.0)
    levels = []
    cor = [None]
    li = 0
    while True:
        M = len(sizes)
        small = top_dense > 0 and sum(sizes) <= top_dense
        if M == 1 or small or all(len(graph[p]) == M - 1 for p in range(M)):
            D = _dense_active(blocks, sizes)
            Ltop = chol_lower(D, li, -1)
            flops["top"] += D.shape[0] ** 3 / 3.0
            return Factor(tree, tol, tol_mode, gemm_prec, levels, list(sizes),
                          [list(g) for g in graph], Ltop, flops, cor[0], dc)
        if level_hook is not None:
            level_hook(li, blocks, sizes, graph)
        rec, cur = _eliminate_level(li, blocks, sizes, graph, tol, tol_mode, gemm_prec,
                                    flops, checks, cor, dc)
        levels.append(rec)
        blocks, sizes, graph = _coarsen(blocks, cur, M)
        li += 1


def solve(F: Factor, b: np.ndarray) -> np.ndarray:
    """Algorithm 2: ``x = M^{-1} b`` for one right-hand side."""
    b = np.asarray(b, dtype=np.float64)
    vec = {c: b[d].copy() for c, d in enumerate(F.tree.leaf_dofs)}
    saved = []
    for lev in F.levels:  # forward substitution
        for r in lev.recs:
            if r.Fc is None:
                y = _lsolve(r.G, vec[r.s])  # S_s
                y = apply_qt(r.V, r.tau, y) if r.k else y  # E_s
            else:  # without deferred compression: rotate, then the fine solve
                y = apply_qt(r.V, r.tau, vec[r.s]) if r.k else vec[r.s].copy()
                y[r.k:] = _lsolve(r.G, y[r.k:])
                y[:r.k] -= r.Fc.T @ y[r.k:]
            yf = y[r.k:]
            off = 0
            for q, wq in r.nlist:  # G_s: y_n -= F^T y_f
                vec[q][:wq] -= r.F[:, off:off + wq].T @ yf
                off += wq
            vec[r.s] = y
        saved.append(vec)
        M = len(lev.sizes)
        vec = {c: np.concatenate([vec[2 * c][:lev.ranks[2 * c]],
                                  vec[2 * c + 1][:lev.ranks[2 * c + 1]]]) for c in range(M // 2)}
    z = np.concatenate([vec[c] for c in range(len(F.top_sizes))]) if F.top_sizes else np.zeros(0)
    z = _ltsolve(F.top_L, _lsolve(F.top_L, z))
    off = np.concatenate([[0], np.cumsum(F.top_sizes)]).astype(int)
    xc = {c: z[off[c]:off[c + 1]] for c in range(len(F.top_sizes))}
    for li in reversed(range(len(F.levels))):  # backward substitution
        lev = F.levels[li]
        vec = saved[li]
        for c in range(len(lev.sizes) // 2):
            kl = lev.ranks[2 * c]
            vec[2 * c][:kl] = xc[c][:kl]
            vec[2 * c + 1][:lev.ranks[2 * c + 1]] = xc[c][kl:]
        for r in reversed(lev.recs):
            x = vec[r.s].copy()
            off = 0
            for q, wq in r.nlist:  # G_s^T: x_f -= F x_n
                x[r.k:] -= r.F[:, off:off + wq] @ vec[q][:wq]
                off += wq
            if r.Fc is None:
                x = apply_q(r.V, r.tau, x) if r.k else x  # E_s^T
                vec[r.s] = _ltsolve(r.G, x)  # S_s^T
            else:
                x[r.k:] = _ltsolve(r.G, x[r.k:] - r.Fc @ x[:r.k])
                vec[r.s] = apply_q(r.V, r.tau, x) if r.k else x
        xc = vec
    out = np.empty_like(b)
    for c, d in enumerate(F.tree.leaf_dofs):
        out[d] = xc[c]
    return out
