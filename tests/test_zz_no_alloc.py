"""lrsp_pcg_noalloc (work vectors in the library's static device array)
against lrsp_pcg (work vectors allocated with the factor), through the C-ABI.

The two run the same kernels in the same order on the same inputs, so
iterates, iteration counts and residuals must agree bit for bit; two calls
in a row on different systems, the second smaller than the first, check that
nothing the first call left in the shared array leaks into the second.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle
from synth import config, lognormal_field, rhs, slab_scalar

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


def _system(L, torch, pr, leaf, tol, nrhs):
    A = L.DeviceMatrix.from_problem(pr)
    F = L.Factor(A, L.Tree(pr.grid, leaf), tol)
    b = np.stack([rhs(pr.n, 20 + j) for j in range(nrhs)], axis=1)
    return A, F, torch.from_numpy(b).cuda()


def test_pcg_noalloc_matches_pcg(torch, L):
    cases = [("slab64", config("slab64"), 256, 1e-2, 2),
             ("slab 24x20x8", slab_scalar(24, 20, 8, 1e4, lognormal_field((20, 24, 8), seed=5)), 64, 1e-3, 1),
             ("slab64 again", config("slab64"), 256, 1e-2, 1)]
    for name, pr, leaf, tol, nrhs in cases:
        _say(f"[noalloc pcg] {name}: n={pr.n}, {nrhs} rhs")
        A, F, b = _system(L, torch, pr, leaf, tol, nrhs)
        x0, it0, rr0 = L.pcg(A, F, b, rtol=1e-8)
        x1, it1, rr1 = L.pcg(A, F, b, rtol=1e-8, noalloc=True)
        torch.cuda.synchronize()
        _say(f"  iters {it1.tolist()} (allocating path {it0.tolist()}), relres {rr1.tolist()}")
        assert np.array_equal(it0, it1) and np.array_equal(rr0, rr1)
        assert torch.equal(x0, x1)
        assert (rr1 <= 1e-8).all()
        if name == "slab 24x20x8":
            # and against the oracle's PCG (iterations within one, residual)
            Fo = oracle.factor(pr.rowptr, pr.col, pr.val, oracle.build_tree(pr.grid, leaf), tol)
            As = pr.scipy()
            bb = b[:, 0].cpu().numpy() if b.dim() == 2 else b.cpu().numpy()
            _, ito, _, ok = oracle.pcg(lambda v: As @ v, bb, lambda r: oracle.solve(Fo, r), 1e-8)
            assert ok and abs(int(it1[0]) - ito) <= 1


def test_pcg_noalloc_rejects_oversize(torch, L):
    pr = slab_scalar(8, 8, 4, 1e3)
    A, F, b = _system(L, torch, pr, 16, 1e-2, 1)
    csr = A.csr()
    csr.n = L.PCG_NOALLOC_MAX_N + 1  # checked before anything is launched
    it = (C.c_int32 * 1)()
    rr = (C.c_double * 1)()
    x = torch.empty_like(b[:, 0])
    st = L.lib().lrsp_pcg_noalloc(C.byref(csr), F.handle, b.data_ptr(), x.data_ptr(), 1, 1e-8, 100, it, rr,
                                  L._stream(None))
    assert st == L.ERR_ARG
    assert b"static work area" in L.lib().lrsp_last_error_info()
