"""Right-preconditioned restarted GMRES through the C-ABI against the oracle.

The paper's Krylov wrapper: GMRES(200), tolerance 1e-12, at most 1000
iterations, the factor as right preconditioner.  Bars: the iteration count
is within one of the oracle's GMRES with the oracle's factor (the GPU
orthogonalises by classical Gram-Schmidt applied twice, the oracle by
modified Gram-Schmidt: equal in exact arithmetic), the run converges and
the true relative residual is at most 1e-11 (the least-squares estimate
stops at 1e-12; the true residual adds the rounding of the last update).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle.gmres import gmres as ogmres
from synth import config, laplace2d, lognormal_field, rhs, slab_scalar, slab_vector

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def L():
    from paper_1811_11248_amd import lrsp
    return lrsp


CASES = {
    "laplace64": (lambda: config("laplace64"), 64, 1e-2),
    "slab_ragged": (lambda: slab_scalar(13, 11, 5, 1e3, lognormal_field((11, 13, 5), seed=2)), 40, 1e-2),
    "vector_m160": (lambda: slab_vector(16, 16, 20, 1e4), 256, 1e-2),
    "slab64": (lambda: config("slab64"), 256, 1e-2),
    "laplace64_loose": (lambda: config("laplace64"), 64, 1e-1),
}


@pytest.mark.parametrize("restart", [200, 3])
@pytest.mark.parametrize("name", list(CASES))
def test_gmres_matches_oracle(torch, L, name, restart):
    mk, leaf, tol = CASES[name]
    pr = mk()
    Fo = oracle.factor(pr.rowptr, pr.col, pr.val, oracle.build_tree(pr.grid, leaf), tol)
    As = pr.scipy()
    b = rhs(pr.n, 0)
    _, ito, rro, ok = ogmres(lambda v: As @ v, b, lambda r: oracle.solve(Fo, r), 1e-12, restart=restart)
    assert ok
    A = L.DeviceMatrix.from_problem(pr)
    F = L.Factor(A, L.Tree(pr.grid, leaf), tol)
    x, it, rr = L.gmres(A, F, torch.from_numpy(b).cuda(), rtol=1e-12, restart=restart)
    _say(f"[gmres {name} restart {restart}] iters gpu {it[0]} oracle {ito}; true relres gpu {rr[0]:.2e} "
         f"oracle {rro:.2e}")
    assert abs(int(it[0]) - ito) <= 1
    assert rr[0] <= 1e-11
    res = np.linalg.norm(b - As @ x.cpu().numpy()) / np.linalg.norm(b)
    assert res <= 1e-11


def test_gmres_two_columns_and_errors(torch, L):
    pr = laplace2d(16)
    A = L.DeviceMatrix.from_problem(pr)
    F = L.Factor(A, L.Tree(pr.grid, 16), 1e-2)
    B = np.stack([rhs(pr.n, 3), rhs(pr.n, 4)], axis=1)
    X, it, rr = L.gmres(A, F, torch.from_numpy(B).cuda())
    for c in range(2):
        x1, it1, _ = L.gmres(A, F, torch.from_numpy(B[:, c].copy()).cuda())
        assert it1[0] == it[c] and torch.equal(x1, X[:, c].contiguous())
    assert (rr <= 1e-11).all()
    with pytest.raises(L.LrspError) as ex:
        L.gmres(A, F, torch.from_numpy(B[:, 0].copy()).cuda(), restart=0)
    assert ex.value.status == L.ERR_ARG
    # a cap of one iteration: not converged, reported as such
    _, it, rr = L.gmres(A, F, torch.from_numpy(B[:, 0].copy()).cuda(), maxit=1, raise_no_conv=False)
    assert it[0] == 1 and rr[0] > 1e-12
