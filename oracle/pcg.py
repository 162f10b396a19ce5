"""Preconditioned conjugate gradients (oracle).

The paper wraps the factor in right-preconditioned GMRES(200) at 1e-12
(Numerical Results, test problems).  The factor here is symmetric by
construction, so the path uses PCG: ``x0 = 0``, recursive residual, stop when
``||r||_2 <= rtol ||b||_2`` or after ``maxit`` iterations.  The iteration
count is the number of matrix-vector products.
"""
from __future__ import annotations

import numpy as np


def pcg(matvec, b, prec=None, rtol=1e-8, maxit=1000):
    """Returns ``(x, iters, true_relres, converged)``."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return x, 0, 0.0, True
    M = prec if prec is not None else (lambda v: v.copy())
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    conv = False
    while it < maxit:
        q = matvec(p)
        alpha = rz / float(p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if float(np.linalg.norm(r)) <= rtol * nb:
            conv = True
            break
        z = M(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    relres = float(np.linalg.norm(b - matvec(x))) / nb
    return x, it, relres, conv
