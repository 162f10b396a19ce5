"""Pins of the oracle's right-preconditioned restarted GMRES.

Against what the mathematics fixes: finite termination in as many steps as
the operator has distinct eigenvalues, one step with an exact
preconditioner, the minimal-residual property (the residual after k steps
equals the least-squares minimum over the Krylov space, computed here by
brute force from an explicit Krylov matrix), restarts that still converge,
and scipy's GMRES on the same system without preconditioning.
"""
import numpy as np
import pytest
import scipy.sparse.linalg

from oracle import build_tree, factor, solve
from oracle.gmres import gmres
from synth import laplace2d, lognormal_field, rhs, slab_scalar


def test_finite_termination():
    d = np.repeat([1.0, 5.0, 20.0, 30.0], 6)
    b = rhs(len(d), 4)
    _, it, rr, ok = gmres(lambda v: d * v, b, None, 1e-12)
    assert ok and it == 4 and rr <= 1e-12


def test_exact_preconditioner_one_step():
    pr = laplace2d(12)
    A = pr.scipy()
    Ad = A.toarray()
    b = rhs(pr.n, 5)
    _, it, rr, ok = gmres(lambda v: A @ v, b, lambda r: np.linalg.solve(Ad, r), 1e-12)
    assert ok and it == 1 and rr <= 1e-12


@pytest.mark.parametrize("use_prec", [False, True])
def test_minimal_residual_property(use_prec):
    # a nonsymmetric operator (GMRES does not rely on symmetry) and, as
    # preconditioner, a diagonal scaling
    rng = np.random.default_rng(7)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    Mi = np.diag(1.0 / np.linspace(1, 3, n)) if use_prec else np.eye(n)
    b = rng.standard_normal(n)
    hist = []
    gmres(lambda v: A @ v, b, lambda r: Mi @ r, 1e-14, restart=200, maxit=12, history=hist)
    AM = A @ Mi
    K = [b / np.linalg.norm(b)]
    for k in range(1, 13):
        # brute force: min over y of ||b - A M^{-1} K_k y||, K_k = [b, AM b, ...]
        Kk = np.stack(K, axis=1)
        y, *_ = np.linalg.lstsq(AM @ Kk, b, rcond=None)
        best = np.linalg.norm(b - AM @ Kk @ y) / np.linalg.norm(b)
        assert abs(hist[k - 1] - best) <= 1e-8 * max(best, 1e-12), k
        v = AM @ K[-1]
        K.append(v / np.linalg.norm(v))


def test_restart_still_converges_and_costs_more():
    pr = laplace2d(16)
    A = pr.scipy()
    b = rhs(pr.n, 6)
    _, it_full, rr_full, ok_full = gmres(lambda v: A @ v, b, None, 1e-10, restart=200)
    _, it_r, rr_r, ok_r = gmres(lambda v: A @ v, b, None, 1e-10, restart=10)
    assert ok_full and ok_r and rr_full <= 1e-10 and rr_r <= 1e-10
    assert it_r >= it_full
    # scipy's GMRES, restart 200, no preconditioner: same iteration count
    count = [0]
    scipy.sparse.linalg.gmres(A, b, rtol=1e-10, atol=0.0, restart=200, maxiter=1,
                              callback=lambda rk: count.__setitem__(0, count[0] + 1), callback_type="pr_norm")
    assert abs(it_full - count[0]) <= 1


def test_with_the_hierarchical_factor():
    # the paper's use: the factor as right preconditioner, 1e-12
    pr = slab_scalar(12, 10, 6, 1e4, lognormal_field((10, 12, 6), seed=4))
    F = factor(pr.rowptr, pr.col, pr.val, build_tree(pr.grid, 48), 1e-2)
    A = pr.scipy()
    b = rhs(pr.n, 0)
    x, it, rr, ok = gmres(lambda v: A @ v, b, lambda r: solve(F, r), 1e-12)
    assert ok and rr <= 1e-11
    _, it0, _, _ = gmres(lambda v: A @ v, b, None, 1e-12, maxit=1000)
    assert it < it0 / 4
