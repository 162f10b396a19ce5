"""Whole-factor pins of the oracle (Algorithms 1 and 2) and of its PCG."""
import numpy as np
import pytest
import scipy.sparse.linalg

from oracle import build_tree, factor, pcg, solve
from synth import config, laplace2d, lognormal_field, rhs, slab_scalar, slab_vector

SMALL = [
    (lambda: laplace2d(8), 8),
    (lambda: laplace2d(16), 16),
    (lambda: laplace2d(16, eps=1e-2), 8),
    (lambda: slab_scalar(8, 8, 4, 1e3, lognormal_field((8, 8, 4), seed=3)), 16),
    (lambda: slab_vector(6, 6, 3, 1e2), 16),
]


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_exact_without_truncation(case):
    # tol = 0 keeps every nonzero pivot: the factor is an exact (sparse,
    # block) Cholesky factorization and M^{-1} b equals A^{-1} b
    mk, leaf = SMALL[case]
    pr = mk()
    T = build_tree(pr.grid, leaf)
    F = factor(pr.rowptr, pr.col, pr.val, T, 0.0)
    b = rhs(pr.n, 1)
    x = solve(F, b)
    xe = np.linalg.solve(pr.scipy().toarray(), b)
    assert np.linalg.norm(x - xe) <= 1e-10 * np.linalg.norm(xe)


def test_four_cluster_strip_is_exact_for_any_tol():
    # a strip of <= 4 clusters produces no far-field fill under the
    # (colour, index) order 0,3,1,2: every step is plain block Cholesky
    # (A_sw = 0 case of the Scaled Low-rank Elimination section)
    pr = laplace2d(32, 2)
    T = build_tree(pr.grid, 16)
    assert T.nleaves == 4
    F = factor(pr.rowptr, pr.col, pr.val, T, 0.5)
    assert F.levels[0].order == [0, 3, 1, 2]
    assert all(k == 0 for k in F.levels[0].ranks)
    b = rhs(pr.n, 2)
    A = pr.scipy()
    x, it, rr, ok = pcg(lambda v: A @ v, b, lambda r: solve(F, r), 1e-8)
    assert ok and it == 1


@pytest.mark.parametrize("tol", [1e-1, 1e-2])
def test_spd_asserted_at_every_level(tol):
    # deferred compression: every diagonal-block Cholesky succeeds, the
    # active matrix after each level is SPD on these inputs, and each
    # compression keeps the ww block SPD (Corollary)
    for pr, leaf in ((laplace2d(16), 8), (slab_scalar(8, 8, 4, 1e4, lognormal_field((8, 8, 4))), 16)):
        T = build_tree(pr.grid, leaf)
        F = factor(pr.rowptr, pr.col, pr.val, T, tol, checks=True)
        for lv in F.levels:
            assert lv.min_eig is None or lv.min_eig > 0
        assert F.corollary_min is None or F.corollary_min > 0


def test_pcg_converges_on_laplace64():
    pr = config("laplace64")
    T = build_tree(pr.grid, pr.leaf)
    F = factor(pr.rowptr, pr.col, pr.val, T, pr.tol)
    A = pr.scipy()
    b = rhs(pr.n, 0)
    x, it, rr, ok = pcg(lambda v: A @ v, b, lambda r: solve(F, r), 1e-8)
    assert ok and rr <= 1e-8
    _, it0, _, _ = pcg(lambda v: A @ v, b, None, 1e-8, 3000)
    assert it < it0 / 5  # the factor is a useful preconditioner
    # the compressed factor is symmetric positive definite as an operator
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal(pr.n), rng.standard_normal(pr.n)
    assert abs(u @ solve(F, v) - v @ solve(F, u)) <= 1e-10 * abs(u @ solve(F, u))


def test_pcg_textbook_cases():
    # M = I on a matrix with 3 distinct eigenvalues: CG ends in 3 steps
    d = np.repeat([1.0, 5.0, 20.0], 7)
    b = rhs(len(d), 4)
    _, it, rr, ok = pcg(lambda v: d * v, b, None, 1e-10)
    assert ok and it == 3
    # exact preconditioner: one step
    pr = laplace2d(12)
    A = pr.scipy()
    Ad = A.toarray()
    _, it, rr, ok = pcg(lambda v: A @ v, b[:0].tolist() or rhs(pr.n, 5),
                        lambda r: np.linalg.solve(Ad, r), 1e-8)
    assert ok and it == 1
    # same iteration count as scipy's CG under the same stopping rule (+-1)
    bb = rhs(pr.n, 6)
    _, it, _, ok = pcg(lambda v: A @ v, bb, None, 1e-8)
    count = [0]
    scipy.sparse.linalg.cg(A, bb, rtol=1e-8, maxiter=1000,
                           callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert ok and abs(it - count[0]) <= 1


def test_top_dense_threshold():
    # "small enough" as a size: the recursion stops at the first level with at
    # most top_dense unknowns; that remainder is factored exactly, so with a
    # threshold covering everything the factor is plain Cholesky (a dense
    # solve at any tol), and a smaller threshold only cuts levels off the end
    pr = slab_scalar(8, 8, 4, 1e3, lognormal_field((8, 8, 4), seed=3))
    T = build_tree(pr.grid, 16)
    b = rhs(pr.n, 1)
    xe = np.linalg.solve(pr.scipy().toarray(), b)
    F = factor(pr.rowptr, pr.col, pr.val, T, 0.5, top_dense=pr.n)
    assert len(F.levels) == 0 and F.top_sizes == [16] * 16
    assert np.linalg.norm(solve(F, b) - xe) <= 1e-10 * np.linalg.norm(xe)
    F0 = factor(pr.rowptr, pr.col, pr.val, T, 1e-1)
    sizes = [sum(lv.sizes) for lv in F0.levels]
    thr = sizes[1]  # the unknowns at the start of level 1
    F1 = factor(pr.rowptr, pr.col, pr.val, T, 1e-1, top_dense=thr)
    assert len(F1.levels) == 1 and sum(F1.top_sizes) == thr
    assert F1.levels[0].ranks == F0.levels[0].ranks
