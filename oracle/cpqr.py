"""Rank-revealing compression of the oracle: column-pivoted Householder QR.

The paper compresses the scaled far-field block ``G_s^{-1} A_sw`` as
``U_hat V_hat^T`` with ``U_hat`` orthogonal and the dropped part
``||V_hat_2|| = eps``, naming a rank-revealing QR as one way to get it
(Eqs. offdiag and offdiag_new).  Reading used here:

* Businger-Golub column pivoting: at step ``j`` every remaining column's
  squared norm over rows ``j..m-1`` is recomputed from scratch (no
  downdating) and the pivot is the column of LOWEST original position among
  those whose squared norm is at least ``(1 - TIE) * max`` (``TIE = 1e-10``);
* the reflector maps the pivot column to ``+||x|| e_1`` so that every
  ``R_jj >= 0``; ``beta = sqrt(norm2)`` reuses the pivoting norm;
* the rank ``k`` is the first step ``j`` whose pivot norm satisfies
  ``R_jj <= tol * R_00`` (relative mode) or ``R_jj <= tol`` (absolute
  mode); otherwise ``k = min(m, b)``.  ``k = 0`` when the block is zero.
"""
from __future__ import annotations

import math

import numpy as np

TIE = 1e-10


def householder_nonneg(x: np.ndarray, norm2: float):
    """Reflector ``H = I - tau v v^T`` (``v[0] = 1``) with ``H x = beta e_1``,
    ``beta = sqrt(norm2) >= 0``.  Returns ``(v, tau, beta)``."""
    beta = math.sqrt(norm2)
    v = np.zeros_like(x)
    v[0] = 1.0
    if beta == 0.0:
        return v, 0.0, 0.0
    alpha = float(x[0])
    rest2 = float(np.dot(x[1:], x[1:]))
    # d = alpha - beta and tau = (beta - alpha)/beta, both evaluated without
    # cancellation when alpha > 0 (beta^2 - alpha^2 = rest2)
    if alpha <= 0.0:
        d = alpha - beta
        tau = (beta - alpha) / beta
    else:
        d = -rest2 / (alpha + beta)
        tau = rest2 / (beta * (beta + alpha))
    if d == 0.0:
        return v, 0.0, beta
    v[1:] = x[1:] / d
    return v, tau, beta


def cpqr(B: np.ndarray, tol: float, tol_mode: str = "relative", info: dict | None = None):
    """Truncated column-pivoted QR ``B P = Q R``.

    Returns ``(k, V, tau, R, perm)``: ``V`` is ``m x k`` with the reflector
    vectors (unit leading entry, zeros above), ``tau`` their scalars, ``R``
    the ``k x b`` upper-trapezoidal factor in pivoted column order, and
    ``perm[c]`` the original column at pivoted position ``c``.

    ``info``, if given, receives the pivot norms that decided the rank:
    ``r00``, ``last`` (the last pivot kept, ``R_{k-1,k-1}``, or None) and
    ``stop`` (the pivot norm that ended the QR, or None when all ``min(m, b)``
    steps ran).
    """
    m, b = B.shape
    if info is not None:
        info.update(r00=0.0, last=None, stop=None)
    W = np.array(B, dtype=np.float64, copy=True)
    perm = np.arange(b)
    kmax = min(m, b)
    V = np.zeros((m, kmax))
    tau = np.zeros(kmax)
    r00 = 0.0
    k = kmax
    for j in range(kmax):
        rem = W[j:, j:]
        norm2 = np.einsum("ij,ij->j", rem, rem)
        mx = float(norm2.max())
        cand = np.nonzero(norm2 >= (1.0 - TIE) * mx)[0]
        c = int(cand[np.argmin(perm[j + cand])])
        piv = j + c
        if piv != j:
            W[:, [j, piv]] = W[:, [piv, j]]
            perm[[j, piv]] = perm[[piv, j]]
        rjj = math.sqrt(float(norm2[c]))
        if j == 0:
            r00 = rjj
            if info is not None:
                info["r00"] = rjj
        stop = (rjj <= tol * r00) if tol_mode == "relative" else (rjj <= tol)
        if stop or rjj == 0.0:
            k = j
            if info is not None:
                info["stop"] = rjj
            break
        if info is not None:
            info["last"] = rjj
        v, t, beta = householder_nonneg(W[j:, j], float(norm2[c]))
        if j + 1 < b:
            blk = W[j:, j + 1:]
            blk -= t * np.outer(v, v @ blk)
        W[j, j] = beta
        W[j + 1:, j] = 0.0
        V[j:, j] = v
        tau[j] = t
    R = np.triu(W[:k, :])
    return k, V[:, :k].copy(), tau[:k].copy(), R, perm


def apply_qt(V: np.ndarray, tau: np.ndarray, X: np.ndarray) -> np.ndarray:
    """``Q^T X`` with ``Q = H_0 H_1 ... H_{k-1}``: apply ``H_0`` first."""
    Y = np.array(X, dtype=np.float64, copy=True)
    squeeze = Y.ndim == 1
    if squeeze:
        Y = Y[:, None]
    for j in range(V.shape[1]):
        v = V[j:, j]
        Y[j:] -= tau[j] * np.outer(v, v @ Y[j:])
    return Y[:, 0] if squeeze else Y


def apply_q(V: np.ndarray, tau: np.ndarray, X: np.ndarray) -> np.ndarray:
    """``Q X``: apply ``H_{k-1}`` first."""
    Y = np.array(X, dtype=np.float64, copy=True)
    squeeze = Y.ndim == 1
    if squeeze:
        Y = Y[:, None]
    for j in reversed(range(V.shape[1])):
        v = V[j:, j]
        Y[j:] -= tau[j] * np.outer(v, v @ Y[j:])
    return Y[:, 0] if squeeze else Y
