"""The elimination WITHOUT deferred compression against Proposition 1.

The deferred-compression section gives the error of the approximate Schur
complement of the original scheme in closed form (Eq. err_old): with
``A_sw = U_1 V_1^T + U_2 V_2^T`` and ``U_2 V_2^T`` dropped,
    E_nn = 0,   E_nw = A_ns A_ss^{-1} U_2 V_2^T,
    E_ww = A_ws A_ss^{-1} A_sw - V_1 U_1^T A_ss^{-1} U_1 V_1^T,
with ||E_nw|| <= e ||A_ns|| / sigma_min(A_ss) and
||E_ww|| <= (2 e ||A_sw|| + e^2) / sigma_min(A_ss), e = ||U_2 V_2^T||.
The oracle's step eliminates the fine DoFs and keeps the coarse ones with
their couplings; eliminating those too gives the whole approximate Schur
complement, compared here with the exact one.  Whole factors: exact at
tol = 0 and on a strip without far field, and a working preconditioner.
"""
import numpy as np
import pytest

from oracle import apply_q, build_tree, factor, pcg, solve
from oracle.hsolver import lowrank_elimination_nodc
from synth import laplace2d, lognormal_field, rhs, slab_scalar, slab_vector


def _spd_3x3(ms, mn, mw, rng, cond=1e6):
    n = ms + mn + mw
    X = rng.standard_normal((n, n))
    X[ms + mn:] *= np.logspace(0, -6, n)[None, :]
    X[:ms, ms // 2:] *= 1e-3
    A = X @ X.T + (1.0 / cond) * np.eye(n)
    return A, slice(0, ms), slice(ms, ms + mn), slice(ms + mn, n)


@pytest.mark.parametrize("seed,tol", [(0, 1e-2), (1, 3e-2), (2, 1e-1), (3, 1e-3)])
def test_proposition1_identities_and_bounds(seed, tol):
    rng = np.random.default_rng(seed)
    ms = 10
    A, s, n, w = _spd_3x3(ms, 8, 14, rng)
    Ass, Asn, Asw = A[s, s], A[s, n], A[s, w]
    st = lowrank_elimination_nodc(Ass, Asn, Asw, tol)
    k = st.k
    assert 0 < k < ms
    U = apply_q(st.V, st.tau, np.eye(ms))
    np.testing.assert_allclose(U.T @ U, np.eye(ms), atol=1e-13)
    U1 = U[:, :k]
    # V_1^T is the coupling of the coarse directions: U_1 V_1^T = U_1 U_1^T A_sw
    np.testing.assert_allclose(U1 @ st.Vt, U1 @ (U1.T @ Asw), atol=1e-13 * np.abs(Asw).max())
    D2 = Asw - U1 @ st.Vt  # U_2 V_2^T, the dropped part
    eps = np.linalg.norm(D2, 2)
    # the rank rule: the first pivot not kept is at most tol times the first
    assert eps <= np.sqrt(Asw.shape[1] - k) * tol * np.linalg.norm(Asw, 2) * 1.0001
    # remaining system after the fine elimination: coarse rows (Dc, Ccn, V1^T)
    # and the near field updated by -Fn^T Fn; eliminate the coarse DoFs too
    nn, nw = A[n, n] - st.Fn.T @ st.Fn, A[n, w]
    X = np.block([[nn, nw], [nw.T, A[w, w]]])
    Cr = np.hstack([st.Ccn, st.Vt])
    S_tilde = X - Cr.T @ np.linalg.solve(st.Dc, Cr)
    # exact Schur complement of s
    B = np.hstack([Asn, Asw])
    S_A = np.block([[A[n, n], A[n, w]], [A[w, n], A[w, w]]]) - B.T @ np.linalg.solve(Ass, B)
    E = S_tilde - S_A
    a = Asn.shape[1]
    Ainv = np.linalg.inv(Ass)
    E_nw = A[n, s] @ Ainv @ D2
    E_ww = A[w, s] @ Ainv @ Asw - (U1 @ st.Vt).T @ Ainv @ (U1 @ st.Vt)
    scale = np.abs(S_A).max()
    np.testing.assert_allclose(E[:a, :a], 0.0, atol=1e-9 * scale)
    np.testing.assert_allclose(E[:a, a:], E_nw, atol=1e-9 * scale)
    np.testing.assert_allclose(E[a:, a:], E_ww, atol=1e-9 * scale)
    smin = np.linalg.eigvalsh(Ass).min()
    assert np.linalg.norm(E_nw, 2) <= eps * np.linalg.norm(A[n, s], 2) / smin * (1 + 1e-8)
    assert np.linalg.norm(E_ww, 2) <= (2 * eps * np.linalg.norm(Asw, 2) + eps ** 2) / smin * (1 + 1e-8)


def test_no_far_field_is_block_cholesky():
    rng = np.random.default_rng(4)
    A, s, n, w = _spd_3x3(6, 5, 4, rng)
    st = lowrank_elimination_nodc(A[s, s], A[s, n], np.zeros((6, 0)), 1e-2)
    assert st.k == 0
    np.testing.assert_allclose(st.Fn.T @ st.Fn, A[n, s] @ np.linalg.solve(A[s, s], A[s, n]), atol=1e-10)


SMALL = [
    (lambda: laplace2d(16), 16),
    (lambda: slab_scalar(8, 8, 4, 1e3, lognormal_field((8, 8, 4), seed=3)), 16),
    (lambda: slab_vector(6, 6, 3, 1e2), 16),
]


@pytest.mark.parametrize("case", range(len(SMALL)))
def test_exact_without_truncation(case):
    mk, leaf = SMALL[case]
    pr = mk()
    F = factor(pr.rowptr, pr.col, pr.val, build_tree(pr.grid, leaf), 0.0, dc=False)
    b = rhs(pr.n, 1)
    xe = np.linalg.solve(pr.scipy().toarray(), b)
    assert np.linalg.norm(solve(F, b) - xe) <= 1e-10 * np.linalg.norm(xe)


def test_strip_without_far_field_is_exact():
    pr = laplace2d(32, 2)
    F = factor(pr.rowptr, pr.col, pr.val, build_tree(pr.grid, 16), 0.5, dc=False)
    assert all(k == 0 for k in F.levels[0].ranks)
    b = rhs(pr.n, 2)
    xe = np.linalg.solve(pr.scipy().toarray(), b)
    assert np.linalg.norm(solve(F, b) - xe) <= 1e-10 * np.linalg.norm(xe)


def test_preconditioner_is_symmetric_and_converges():
    pr = slab_scalar(12, 10, 6, 1e2, lognormal_field((10, 12, 6), seed=4))
    F = factor(pr.rowptr, pr.col, pr.val, build_tree(pr.grid, 48), 1e-2, dc=False)
    A = pr.scipy()
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal(pr.n), rng.standard_normal(pr.n)
    assert abs(u @ solve(F, v) - v @ solve(F, u)) <= 1e-10 * abs(u @ solve(F, u))
    b = rhs(pr.n, 0)
    _, it, rr, ok = pcg(lambda x: A @ x, b, lambda r: solve(F, r), 1e-8)
    assert ok and rr <= 1e-8
