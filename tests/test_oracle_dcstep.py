"""One scaled low-rank elimination against Proposition 2 and its Corollary.

The deferred-compression section gives the error of the approximate Schur
complement in closed form (Eq. err_new):
    E_nw = A_ns G^{-T} U2 V2^T,   E_ww = V2 V2^T,   E_nn = 0,
with ||E_ww|| = ||V2||^2 and ||E_nw|| <= ||V2|| ||A_ns|| / sigma_min(A_ss)^{1/2},
and the ww block of the approximate Schur complement stays SPD.
The oracle's step returns G, the reflectors of U_hat, C = U^T G^{-1} A_sn and
V1^T; from those the approximate Schur complement of all of s is rebuilt and
compared with the exact one.
"""
import numpy as np
import pytest

from oracle import apply_q, scaled_lowrank_elimination


def _spd_3x3(ms, mn, mw, rng, cond=1e6):
    # A = X X^T + delta I is SPD; damping the far-field rows of X column by
    # column gives A_sw = X_s X_w^T decaying singular values, and a small
    # delta with a rank-deficient X_s makes A_ss ill-conditioned
    n = ms + mn + mw
    X = rng.standard_normal((n, n))
    X[ms + mn:] *= np.logspace(0, -6, n)[None, :]
    X[:ms, ms // 2:] *= 1e-3
    A = X @ X.T + (1.0 / cond) * np.eye(n)
    s, ns, w = slice(0, ms), slice(ms, ms + mn), slice(ms + mn, n)
    return A, s, ns, w


@pytest.mark.parametrize("seed,tol", [(0, 1e-2), (1, 3e-2), (2, 1e-1)])
def test_proposition2_identities(seed, tol):
    rng = np.random.default_rng(seed)
    A, s, n, w = _spd_3x3(10, 8, 14, rng)
    st = scaled_lowrank_elimination(A[s, s], A[s, n], A[s, w], tol)
    k, ms = st.k, 10
    assert 0 < k < 10
    G = st.G
    np.testing.assert_allclose(G @ G.T, A[s, s], atol=1e-13 * np.abs(A).max())
    C1, F = st.C[:k], st.C[k:]
    # approximate Schur complement of all of s: eliminate the fine DoFs
    # (near field updated by F^T F), then the k coarse DoFs with their
    # identity diagonal block
    S_nn = A[n, n] - F.T @ F - C1.T @ C1
    S_nw = A[n, w] - C1.T @ st.Vt
    S_ww = A[w, w] - st.Vt.T @ st.Vt
    Ainv = np.linalg.inv(A[s, s])
    E_nn = S_nn - (A[n, n] - A[n, s] @ Ainv @ A[s, n])
    E_nw = S_nw - (A[n, w] - A[n, s] @ Ainv @ A[s, w])
    E_ww = S_ww - (A[w, w] - A[w, s] @ Ainv @ A[s, w])
    Uh = apply_q(st.V, st.tau, np.eye(ms))
    U2 = Uh[:, k:]
    V2t = U2.T @ np.linalg.solve(G, A[s, w])
    scale = np.abs(A).max() * np.linalg.cond(A[s, s])
    np.testing.assert_allclose(E_nn, 0, atol=1e-12 * scale)
    np.testing.assert_allclose(E_nw, A[n, s] @ np.linalg.solve(G.T, U2 @ V2t), atol=1e-12 * scale)
    np.testing.assert_allclose(E_ww, V2t.T @ V2t, atol=1e-12 * scale)
    nv2 = np.linalg.norm(V2t, 2)
    assert np.linalg.norm(E_ww, 2) == pytest.approx(nv2 ** 2, rel=1e-6, abs=1e-14)
    smin = np.linalg.svd(A[s, s], compute_uv=False).min()
    assert np.linalg.norm(E_nw, 2) <= nv2 * np.linalg.norm(A[n, s], 2) / np.sqrt(smin) * (1 + 1e-8)
    # ||V2|| is controlled by the truncation rule: <= sqrt(b-k) * tol * R00
    assert nv2 <= np.sqrt(14 - k) * tol * st.R[0, 0] * (1 + 1e-12)
    # Corollary: the ww block is SPD
    assert np.linalg.eigvalsh(S_ww).min() > 0


def test_no_far_field_is_block_cholesky():
    # A_sw = 0 reduces the step to plain block Cholesky (k = 0, F = G^{-1} A_sn)
    rng = np.random.default_rng(9)
    A, s, n, w = _spd_3x3(6, 5, 4, rng, cond=1e3)
    st = scaled_lowrank_elimination(A[s, s], A[s, n], np.zeros((6, 0)), 1e-2)
    assert st.k == 0
    S = A[n, n] - st.C.T @ st.C
    np.testing.assert_allclose(S, A[n, n] - A[n, s] @ np.linalg.solve(A[s, s], A[s, n]), atol=1e-12)
    st = scaled_lowrank_elimination(A[s, s], A[s, n], np.zeros((6, 3)), 1e-2)
    assert st.k == 0
