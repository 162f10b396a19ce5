"""Pins of the oracle's rank-revealing compression (column-pivoted QR)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import apply_q, apply_qt, cpqr, householder_nonneg


def _q(V, tau, m):
    return apply_q(V, tau, np.eye(m))


@pytest.mark.parametrize("x", [
    np.array([3.0, 4.0, 0.0]), np.array([-3.0, 4.0, 12.0]), np.array([2.0, 0.0, 0.0]),
    np.array([-2.0, 0.0]), np.array([1e-3, -5.0, 2.0, 7.0]),
    np.array([1.0, 1e-9, 0.0]), np.array([1.0, -3e-12, 2e-12])])
def test_householder_maps_to_nonnegative_axis(x):
    v, tau, beta = householder_nonneg(x, float(x @ x))
    H = np.eye(len(x)) - tau * np.outer(v, v)
    e = np.zeros_like(x)
    e[0] = np.linalg.norm(x)
    np.testing.assert_allclose(H @ x, e, atol=1e-14 * np.linalg.norm(x))
    np.testing.assert_allclose(H @ H.T, np.eye(len(x)), atol=1e-14)
    assert beta >= 0 and v[0] == 1.0


@pytest.mark.parametrize("shape", [(12, 9), (9, 12), (20, 20), (30, 7)])
def test_pivots_match_lapack_on_generic_matrices(shape):
    # for a generic matrix (no ties) the Businger-Golub pivot sequence is
    # the one LAPACK's xGEQP3 takes; R agrees up to the sign of each row
    rng = np.random.default_rng(sum(shape))
    B = rng.standard_normal(shape)
    k, V, tau, R, perm = cpqr(B, 0.0)
    Rl, pl = scipy.linalg.qr(B, pivoting=True, mode="r")
    assert k == min(shape)
    assert np.array_equal(perm[:k], pl[:k])
    np.testing.assert_allclose(np.abs(R), np.abs(Rl[:k]), atol=1e-12 * np.abs(Rl).max())
    assert np.all(np.diag(R) >= 0)


def test_factorisation_identity_and_truncation_bound():
    rng = np.random.default_rng(3)
    m, b = 25, 40
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    W, _ = np.linalg.qr(rng.standard_normal((b, m)))
    s = 10.0 ** -np.linspace(0, 8, m)
    B = U @ np.diag(s) @ W.T
    for tol in (1e-1, 1e-3, 1e-6):
        k, V, tau, R, perm = cpqr(B, tol)
        Q = _q(V, tau, m)
        np.testing.assert_allclose(Q.T @ Q, np.eye(m), atol=1e-13)
        # B P = Q [R; R22]: the first k rows are R
        QtB = Q.T @ B[:, perm]
        np.testing.assert_allclose(np.triu(QtB[:k]), R, atol=1e-13)
        np.testing.assert_allclose(QtB[:k][np.tril_indices(k, -1)], 0, atol=1e-13)
        d = np.abs(np.diag(R))
        assert np.all(np.diff(d) <= 1e-15 * d[0])  # non-increasing
        assert d[k - 1] > tol * d[0]
        # the dropped block: its largest column norm is the next pivot,
        # which is <= tol*R00; sigma_{k+1}(B) <= ||R22|| <= sqrt(b-k)*tol*R00
        R22 = QtB[k:, k:]
        assert np.linalg.norm(R22, axis=0).max() <= tol * d[0] * (1 + 1e-12)
        assert s[k] <= np.sqrt(b - k) * tol * d[0] * (1 + 1e-12)
        # apply_qt is the transpose of apply_q
        X = rng.standard_normal((m, 3))
        np.testing.assert_allclose(apply_qt(V, tau, X), Q.T @ X, atol=1e-13)


def test_brute_force_pivots_with_ties():
    # exact ties: columns 1 and 3 are copies; brute force picks the lowest
    # original position among the largest norms at every step
    rng = np.random.default_rng(5)
    c = rng.standard_normal(6)
    B = np.stack([0.5 * c, c, rng.standard_normal(6) * 0.1, c, 0.3 * rng.standard_normal(6)], 1)
    k, V, tau, R, perm = cpqr(B, 0.0)
    W = B.copy()
    rem = list(range(B.shape[1]))
    Q = np.eye(6)
    for j in range(k):
        Z = Q.T @ W
        norms = {col: float(Z[j:, col] @ Z[j:, col]) for col in rem}
        mx = max(norms.values())
        best = min(col for col in rem if norms[col] >= (1 - 1e-10) * mx)
        assert perm[j] == best
        rem.remove(best)
        Q = _q(V[:, :j + 1], tau[:j + 1], 6)


def test_zero_block_has_rank_zero():
    k, V, tau, R, perm = cpqr(np.zeros((5, 4)), 1e-2)
    assert k == 0 and R.shape == (0, 4)


def test_absolute_mode():
    B = np.diag([4.0, 2.0, 1.0, 0.5])
    assert cpqr(B, 0.6, "absolute")[0] == 3
    assert cpqr(B, 0.3, "relative")[0] == 2  # 1.0 <= 0.3*4
