"""Right-preconditioned restarted GMRES (oracle).

The paper solves its systems with right-preconditioned restarted GMRES(200)
(Trilinos Belos), stopping at a relative residual of 1e-12 or after 1000
iterations (Numerical Results, test problems).  This is that iteration
written out in its textbook form (Saad, "Iterative Methods for Sparse Linear
Systems", Algorithms 6.9 and 9.5): with ``x0 = 0`` and the preconditioner
``M``, each cycle builds an orthonormal basis ``V`` of the Krylov space of
``A M^{-1}`` from ``r0 = b - A x0`` by modified Gram-Schmidt, reduces the
Hessenberg matrix with Givens rotations, and stops when the least-squares
residual ``|g_{j+1}|`` falls to ``rtol ||b||``; the iterate is then
``x = x0 + M^{-1} V y``.  The iteration count is the number of products
with ``A M^{-1}`` over all cycles.
"""
from __future__ import annotations

import math

import numpy as np


def _givens(a: float, b: float):
    """(c, s) with [c s; -s c] [a; b] = [r; 0], r >= 0 when b != 0."""
    if b == 0.0:
        return 1.0, 0.0
    r = math.hypot(a, b)
    return a / r, b / r


def gmres(matvec, b, prec=None, rtol=1e-12, restart=200, maxit=1000, history=None):
    """Returns ``(x, iters, true_relres, converged)``.

    history, if a list, receives the residual estimate |g_{j+1}| / ||b||
    after every Arnoldi step."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return x, 0, 0.0, True
    M = prec if prec is not None else (lambda v: v.copy())
    it = 0
    conv = False
    while it < maxit and not conv:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        if beta <= rtol * nb:
            conv = True
            break
        m = min(restart, maxit - it)
        V = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(m):
            w = matvec(M(V[:, j]))
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = float(V[:, i] @ w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0.0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):  # earlier rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            if history is not None:
                history.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= rtol * nb or H[j, j] == 0.0:
                conv = abs(g[j + 1]) <= rtol * nb
                break
        k = j_done
        y = np.zeros(k)
        for i in reversed(range(k)):  # back substitution with the rotated H
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + M(V[:, :k] @ y)
    relres = float(np.linalg.norm(b - matvec(x))) / nb
    return x, it, relres, conv
