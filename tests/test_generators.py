"""Pins of the seeded input generators."""
import numpy as np
import pytest

from synth import batch_params, config, laplace2d, lognormal_field, slab_scalar, slab_vector


@pytest.mark.parametrize("n", [8, 16])
@pytest.mark.parametrize("eps", [1.0, 1e-2])
def test_laplace_eigenvalues_closed_form(n, eps):
    # Introduction: the 5-point discretisation of eps*u_xx + u_yy on an n x n
    # grid has eigenvalues 4(n+1)^2 [eps sin^2(pi i/(2n+2)) + sin^2(pi j/(2n+2))].
    A = laplace2d(n, eps=eps).scipy().toarray()
    ev = np.sort(np.linalg.eigvalsh(A))
    i, j = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1))
    cf = 4 * (n + 1) ** 2 * (eps * np.sin(np.pi * i / (2 * n + 2)) ** 2
                             + np.sin(np.pi * j / (2 * n + 2)) ** 2)
    cf = np.sort(cf.ravel())
    assert np.max(np.abs(ev - cf)) <= 1e-12 * cf.max()


def test_config_sizes():
    p = config("laplace64")
    assert (p.n, p.nnz, p.leaf, p.tol) == (4096, 20224, 64, 1e-2)
    p = config("slab64")
    assert (p.n, p.nnz, p.leaf) == (65536, 446464, 256)
    A = p.scipy()
    assert abs(A - A.T).max() == 0.0


def test_slab_row_sums_are_boundary_terms():
    # With kappa = 1, interior faces cancel in A*1; what is left is the
    # Dirichlet half-cell term 2*kappa*factor on lateral (factor 1) and
    # bottom (factor ratio) faces, nothing on the Neumann top.
    nx, ny, nz, ratio = 5, 4, 3, 100.0
    A = slab_scalar(nx, ny, nz, ratio).scipy()
    s = A @ np.ones(A.shape[0])
    exp = np.zeros((ny, nx, nz))
    exp[:, 0, :] += 2
    exp[:, -1, :] += 2
    exp[0, :, :] += 2
    exp[-1, :, :] += 2
    exp[:, :, 0] += 2 * ratio
    np.testing.assert_allclose(s, exp.ravel(), rtol=1e-13, atol=1e-12)
    # vertical coupling = ratio * harmonic mean, horizontal = harmonic mean
    kap = lognormal_field((ny, nx, nz), seed=7)
    A = slab_scalar(nx, ny, nz, ratio, kap).scipy()
    cell = lambda y, x, z: z + nz * (x + nx * y)  # noqa: E731
    hm = 2 * kap[1, 2, 0] * kap[1, 2, 1] / (kap[1, 2, 0] + kap[1, 2, 1])
    assert A[cell(1, 2, 0), cell(1, 2, 1)] == pytest.approx(-ratio * hm, rel=1e-14)
    hm = 2 * kap[1, 2, 0] * kap[1, 3, 0] / (kap[1, 2, 0] + kap[1, 3, 0])
    assert A[cell(1, 2, 0), cell(1, 3, 0)] == pytest.approx(-hm, rel=1e-14)


def test_vector_operator_spd_and_coupling():
    p = slab_vector(4, 3, 3, 1e3)
    A = p.scipy().toarray()
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0
    # x-face between cells (y=0,x=0,z=1) and (y=0,x=1,z=1): -T*M_x, T=1
    a, b = 1 + 3 * 0, 1 + 3 * 1
    np.testing.assert_allclose(A[2 * a:2 * a + 2, 2 * b:2 * b + 2], -np.array([[2, .3], [.3, 1]]))
    # nnz: 4 per diagonal block + 8 per interior face
    faces = 3 * 3 * 3 + 4 * 2 * 3 + 4 * 3 * 2
    assert p.nnz == 4 * 36 + 8 * faces


def test_lognormal_field_statistics():
    k = lognormal_field((32, 32, 8), seed=1)
    g = np.log(k)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1.0) < 1e-12
    # correlated: neighbouring cells are strongly correlated
    assert np.corrcoef(g[:, :-1].ravel(), g[:, 1:].ravel())[0, 1] > 0.8


def test_batch_params_ranges():
    ps = batch_params()
    assert len(ps) == 512
    for p in ps:
        assert 16 <= p["nx"] == p["ny"] <= 48 and 8 <= p["nz"] <= 24
        assert 1e2 <= p["ratio"] <= 1e5
    ns = [p["nx"] * p["ny"] * p["nz"] for p in ps]
    assert min(ns) >= 2048 and max(ns) <= 55296


def test_icesheet_slab_boundary_types():
    # homogeneous Neumann on top and lateral faces and a Robin bed that is
    # zero under the floating shelf: constant fields are in the kernel of
    # every row except those of grounded bottom cells, whose row sums are the
    # Robin face term times the vertical coupling matrix
    from synth import slab_icesheet
    from synth.problems import coupling_mats
    nx, ny, nz, ratio, beta = 6, 5, 4, 1e3, 50.0
    kap = lognormal_field((ny, nx, nz), seed=3)
    pr = slab_icesheet(nx, ny, nz, ratio, kap, shelf_frac=0.5, beta=beta)
    A = pr.scipy()
    assert abs(A - A.T).max() == 0.0
    Mz = coupling_mats()[2]
    for comp in range(2):
        e = np.zeros(pr.n)
        e[comp::2] = 1.0
        r = A @ e
        for y in range(ny):
            for x in range(nx):
                for z in range(nz):
                    cid = z + nz * (x + nx * y)
                    want = np.zeros(2)
                    if z == 0 and x < 0.5 * nx:
                        tb = 1.0 / (1.0 / (2.0 * ratio * kap[y, x, 0]) + 1.0 / beta)
                        want = tb * Mz[:, comp]
                    np.testing.assert_allclose(r[2 * cid:2 * cid + 2], want, atol=1e-9 * ratio)
    # SPD, and far more ill-conditioned than the Dirichlet slab
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > 0
    evd = np.linalg.eigvalsh(slab_vector(nx, ny, nz, ratio, kap).scipy().toarray())
    assert ev.max() / ev.min() > 10 * evd.max() / evd.min()
