"""Synthetic SPD test problems that stand in for the paper's ice-sheet systems.

The paper's experiments use Antarctic first-order-Stokes matrices on extruded
meshes (thin slabs, strong vertical and weak horizontal coupling, two unknowns
per mesh node; Numerical Results section).  Those matrices are not available,
so every problem here is synthetic and seeded:

* ``laplace2d``   -- the 5-point finite-difference operator of the model
  problem ``eps*u_xx + u_yy`` quoted in the Introduction (Dirichlet boundary),
  whose eigenvalues are known in closed form.
* ``slab_scalar`` -- a cell-centred 7-point finite-volume diffusion operator on
  an extruded ``nx x ny x nz`` slab: face transmissibility is the harmonic mean
  of the cell conductivities times a direction factor (1 horizontally,
  ``ratio`` vertically); Dirichlet on the lateral and bottom faces (half-cell
  distance, i.e. ``2*kappa``), homogeneous Neumann on the top face, mirroring
  the top-surface boundary condition of the ice-sheet model.
* ``slab_vector`` -- the two-component analogue: every face term is the
  scalar transmissibility times a fixed 2x2 SPD coupling matrix per
  direction, so each per-node block is SPD; a stand-in for the
  two-unknowns-per-node Stokes-like system.

Global DoF numbering keeps every vertical column contiguous:
``id = c + ncomp*(z + nz*(x + nx*y))`` (2-D: ``id = x + nx*y``).

Matrices are returned as CSR with a full symmetric pattern, sorted column
indices, int64 row pointers, int32 columns and float64 values.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.ndimage
import scipy.sparse as sp


@dataclasses.dataclass
class Problem:
    name: str
    grid: tuple  # (nx, ny, nz, ncomp)
    rowptr: np.ndarray  # int64 [n+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]
    leaf: int = 256
    tol: float = 1e-2
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def _to_csr(rows, cols, vals, n):
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    # duplicate sums may round differently in the two triangles; make the
    # stored matrix exactly symmetric
    m = ((m + m.T) * 0.5).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return (m.indptr.astype(np.int64), m.indices.astype(np.int32),
            m.data.astype(np.float64))


def laplace2d(nx: int, ny: int | None = None, eps: float = 1.0) -> Problem:
    """5-point operator of ``eps*u_xx + u_yy`` on the unit square, Dirichlet.

    Interior grid ``nx x ny``, spacing ``h = 1/(nx+1)`` in x and
    ``1/(ny+1)`` in y; DoF ``x + nx*y``.
    """
    ny = nx if ny is None else ny
    hx2 = float(nx + 1) ** 2
    hy2 = float(ny + 1) ** 2
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ids = (x + nx * y).ravel()
    xs = x.ravel()
    ys = y.ravel()
    rows = [ids]
    cols = [ids]
    vals = [np.full(ids.shape, 2.0 * eps * hx2 + 2.0 * hy2)]
    for dx, dy, w in ((1, 0, eps * hx2), (-1, 0, eps * hx2), (0, 1, hy2), (0, -1, hy2)):
        ok = (xs + dx >= 0) & (xs + dx < nx) & (ys + dy >= 0) & (ys + dy < ny)
        rows.append(ids[ok])
        cols.append((xs[ok] + dx) + nx * (ys[ok] + dy))
        vals.append(np.full(int(ok.sum()), -w))
    n = nx * ny
    rp, c, v = _to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)
    return Problem("laplace2d", (nx, ny, 1, 1), rp, c, v,
                   params={"eps": eps})


def lognormal_field(shape, ell: float = 8.0, sigma: float = 1.0, seed: int = 1) -> np.ndarray:
    """kappa = exp(sigma*g), g = standardised Gaussian-smoothed white noise.

    ``shape`` is ``(ny, nx, nz)``; the smoothing kernel has standard
    deviation ``ell/sqrt(2)`` cells in every direction with reflecting
    boundaries.
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(shape)
    g = scipy.ndimage.gaussian_filter(g, sigma=ell / math.sqrt(2.0), mode="reflect")
    g = (g - g.mean()) / g.std()
    return np.exp(sigma * g)


def _faces(nx, ny, nz, kappa, ratio):
    """Yield (cell_a, cell_b, T, direction) for interior faces and
    (cell, T, direction) for Dirichlet boundary faces."""
    cell = lambda y, x, z: z + nz * (x + nx * y)  # noqa: E731
    Y, X, Z = np.meshgrid(np.arange(ny), np.arange(nx), np.arange(nz), indexing="ij")
    hm = lambda a, b: 2.0 * a * b / (a + b)  # noqa: E731
    inner = []
    # x faces
    a = (Y[:, :-1, :], X[:, :-1, :], Z[:, :-1, :])
    inner.append((cell(*a).ravel(), cell(a[0], a[1] + 1, a[2]).ravel(),
                  hm(kappa[:, :-1, :], kappa[:, 1:, :]).ravel(), 0))
    # y faces
    a = (Y[:-1], X[:-1], Z[:-1])
    inner.append((cell(*a).ravel(), cell(a[0] + 1, a[1], a[2]).ravel(),
                  hm(kappa[:-1], kappa[1:]).ravel(), 1))
    # z faces
    a = (Y[:, :, :-1], X[:, :, :-1], Z[:, :, :-1])
    inner.append((cell(*a).ravel(), cell(a[0], a[1], a[2] + 1).ravel(),
                  ratio * hm(kappa[:, :, :-1], kappa[:, :, 1:]).ravel(), 2))
    bnd = []
    for sl, d, f in (((slice(None), 0, slice(None)), 0, 1.0),
                     ((slice(None), nx - 1, slice(None)), 0, 1.0),
                     ((0, slice(None), slice(None)), 1, 1.0),
                     ((ny - 1, slice(None), slice(None)), 1, 1.0),
                     ((slice(None), slice(None), 0), 2, ratio)):
        bnd.append((cell(Y[sl], X[sl], Z[sl]).ravel(), (f * 2.0 * kappa[sl]).ravel(), d))
    return inner, bnd


def slab_scalar(nx: int, ny: int, nz: int, ratio: float, kappa=None) -> Problem:
    """Cell-centred 7-point FV diffusion on an extruded slab (see module doc)."""
    if kappa is None:
        kappa = np.ones((ny, nx, nz))
    inner, bnd = _faces(nx, ny, nz, kappa, ratio)
    n = nx * ny * nz
    rows, cols, vals = [], [], []
    for a, b, t, _ in inner:
        rows += [a, b, a, b]
        cols += [a, b, b, a]
        vals += [t, t, -t, -t]
    for a, t, _ in bnd:
        rows.append(a)
        cols.append(a)
        vals.append(t)
    rp, c, v = _to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)
    return Problem("slab_scalar", (nx, ny, nz, 1), rp, c, v, params={"ratio": ratio})


# 2x2 SPD per-direction coupling matrices of the two-component operator.
def coupling_mats(c: float = 0.3):
    return (np.array([[2.0, c], [c, 1.0]]),
            np.array([[1.0, c], [c, 2.0]]),
            np.array([[1.0, c], [c, 1.0]]))


def slab_vector(nx: int, ny: int, nz: int, ratio: float, kappa=None,
                coupling: float = 0.3) -> Problem:
    """Two-component coupled analogue of ``slab_scalar`` (see module doc)."""
    if kappa is None:
        kappa = np.ones((ny, nx, nz))
    M = coupling_mats(coupling)
    inner, bnd = _faces(nx, ny, nz, kappa, ratio)
    n = 2 * nx * ny * nz
    rows, cols, vals = [], [], []
    for a, b, t, d in inner:
        for ci in range(2):
            for cj in range(2):
                tv = t * M[d][ci, cj]
                ai, aj = 2 * a + ci, 2 * a + cj
                bi, bj = 2 * b + ci, 2 * b + cj
                rows += [ai, bi, ai, bi]
                cols += [aj, bj, bj, aj]
                vals += [tv, tv, -tv, -tv]
    for a, t, d in bnd:
        for ci in range(2):
            for cj in range(2):
                rows.append(2 * a + ci)
                cols.append(2 * a + cj)
                vals.append(t * M[d][ci, cj])
    rp, c, v = _to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)
    return Problem("slab_vector", (nx, ny, nz, 2), rp, c, v,
                   params={"ratio": ratio, "coupling": coupling})


def slab_icesheet(nx: int, ny: int, nz: int, ratio: float, kappa=None, shelf_frac: float = 0.5,
                  beta: float = 1e2, coupling: float = 0.3) -> Problem:
    """Two-component extruded slab with the ice sheet's boundary types.

    The boundary conditions of the first-order Stokes model in the paper's
    Ice Sheet Model section: homogeneous Neumann on the top surface and on
    the lateral (open-ocean) boundary, and a Robin (basal sliding) condition
    on the bottom whose coefficient is ``beta`` where the ice is grounded
    (``x < (1 - shelf_frac) nx``) and zero under the floating shelf.  With a
    floating part the operator is anchored only through the grounded bed, so
    its diagonal blocks are far more ill-conditioned than with Dirichlet
    faces.  Interior faces and coupling matrices as in ``slab_vector``; the
    bottom face term is the series of the half cell (``2 ratio kappa``) and
    the Robin resistance ``1 / beta``.
    """
    if kappa is None:
        kappa = np.ones((ny, nx, nz))
    M = coupling_mats(coupling)
    inner, _ = _faces(nx, ny, nz, kappa, ratio)
    cell = lambda y, x, z: z + nz * (x + nx * y)  # noqa: E731
    Y, X, Z = np.meshgrid(np.arange(ny), np.arange(nx), np.arange(nz), indexing="ij")
    sl = (slice(None), slice(None), 0)
    grounded = X[sl] < (1.0 - shelf_frac) * nx
    kb = kappa[sl]
    tb = np.where(grounded, 1.0 / (1.0 / (2.0 * ratio * kb) + 1.0 / beta), 0.0)
    bnd = [(cell(Y[sl], X[sl], Z[sl]).ravel(), tb.ravel(), 2)]
    n = 2 * nx * ny * nz
    rows, cols, vals = [], [], []
    for a, b, t, d in inner:
        for ci in range(2):
            for cj in range(2):
                tv = t * M[d][ci, cj]
                ai, aj = 2 * a + ci, 2 * a + cj
                bi, bj = 2 * b + ci, 2 * b + cj
                rows += [ai, bi, ai, bi]
                cols += [aj, bj, bj, aj]
                vals += [tv, tv, -tv, -tv]
    for a, t, d in bnd:
        for ci in range(2):
            for cj in range(2):
                rows.append(2 * a + ci)
                cols.append(2 * a + cj)
                vals.append(t * M[d][ci, cj])
    rp, c, v = _to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)
    return Problem("slab_icesheet", (nx, ny, nz, 2), rp, c, v,
                   params={"ratio": ratio, "shelf_frac": shelf_frac, "beta": beta, "coupling": coupling})


def layer_mesh(npts: int, seed: int = 0):
    """Unstructured horizontal layer: ``npts`` random points in an irregular
    sheet-like region (a disk with a bay cut out), numbered in the order they
    were drawn, and the edges of their Delaunay triangulation.  Returns
    ``(xy [npts, 2], adj_ptr, adj)`` with the symmetric, sorted adjacency."""
    import scipy.spatial

    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < npts:
        p = rng.uniform(-1.0, 1.0, size=2)
        r = math.hypot(p[0], p[1])
        bay = math.hypot(p[0] - 0.75, p[1] - 0.1) < 0.45
        if r <= 1.0 and not bay:
            pts.append(p)
    xy = np.array(pts)
    tri = scipy.spatial.Delaunay(xy).simplices
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.concatenate([e, e[:, ::-1]])
    g = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(npts, npts)).tocsr()
    g.sum_duplicates()
    g.sort_indices()
    return xy, g.indptr.astype(np.int64), g.indices.astype(np.int32)


def extruded_mesh(npts: int, nz: int, ratio: float, seed: int = 0, beta: float = 1e2,
                  coupling: float = 0.3) -> Problem:
    """Two-component operator on an unstructured extruded mesh: the layer of
    ``layer_mesh`` repeated over ``nz`` layers.  Horizontal couplings along
    the layer's edges (transmissibility = harmonic mean of a log-normal
    coefficient, times the horizontal 2x2 coupling matrix), vertical
    couplings ``ratio`` times that, Neumann on top and sides and a Robin bed
    with coefficient ``beta`` (grounded everywhere, so the operator is SPD).
    DoF id ``c + 2 (z + nz v)`` for column v.  The layer's graph is returned
    in ``params`` (``layer_adj_ptr``, ``layer_adj``) for the extruded tree."""
    xy, ap, aj = layer_mesh(npts, seed)
    rng = np.random.default_rng(seed + 1)
    # smooth log-normal coefficient: a few Fourier modes in (x, y), a linear
    # trend in z, per-cell noise
    a = rng.standard_normal((3, 2))
    zz = np.arange(nz) / max(1, nz - 1)
    g = (a[0, 0] * np.sin(2.0 * xy[:, 0] + a[0, 1]) + a[1, 0] * np.cos(3.0 * xy[:, 1] + a[1, 1]))[:, None] \
        + a[2, 0] * zz[None, :] + 0.3 * rng.standard_normal((npts, nz))
    kappa = np.exp(g)  # [column, layer]
    Mh = np.array([[1.5, coupling], [coupling, 1.5]])
    Mz = coupling_mats(coupling)[2]
    col = lambda v, z: z + nz * v  # noqa: E731
    rows, cols, vals = [], [], []

    def add(ia, ib, t, M):
        for ci in range(2):
            for cj in range(2):
                tv = t * M[ci, cj]
                rows.extend([2 * ia + ci, 2 * ib + ci, 2 * ia + ci, 2 * ib + ci])
                cols.extend([2 * ia + cj, 2 * ib + cj, 2 * ib + cj, 2 * ia + cj])
                vals.extend([tv, tv, -tv, -tv])

    hm = lambda p, q: 2.0 * p * q / (p + q)  # noqa: E731
    src = np.repeat(np.arange(npts), np.diff(ap))
    up = src < aj  # each edge once
    va, vb = src[up], aj[up].astype(np.int64)
    for z in range(nz):
        add(col(va, z), col(vb, z), hm(kappa[va, z], kappa[vb, z]), Mh)
    for z in range(nz - 1):
        v = np.arange(npts)
        add(col(v, z), col(v, z + 1), ratio * hm(kappa[:, z], kappa[:, z + 1]), Mz)
    tb = 1.0 / (1.0 / (2.0 * ratio * kappa[:, 0]) + 1.0 / beta)
    cb = col(np.arange(npts), 0)
    for ci in range(2):
        for cj in range(2):
            rows.append(2 * cb + ci)
            cols.append(2 * cb + cj)
            vals.append(tb * Mz[ci, cj])
    n = 2 * npts * nz
    rows = [np.asarray(r).ravel() for r in rows]
    cols = [np.asarray(c).ravel() for c in cols]
    vals = [np.asarray(v, dtype=np.float64).ravel() for v in vals]
    rp, c, v = _to_csr(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n)
    return Problem("extruded_mesh", (npts, 1, nz, 2), rp, c, v,
                   params={"ratio": ratio, "beta": beta, "layer_adj_ptr": ap, "layer_adj": aj, "xy": xy})


def rhs(n: int, seed: int = 0) -> np.ndarray:
    """i.i.d. N(0,1) right-hand side."""
    return np.random.default_rng(seed).standard_normal(n)


BATCH_SEED = 4
BATCH_SIZE = 512


def batch_params(nsys: int = BATCH_SIZE, seed: int = BATCH_SEED):
    """Grid draws of the many-systems workload: square horizontal size
    U{16..48}, vertical U{8..24}, vertical/horizontal ratio 10^U(2,5)."""
    rng = np.random.default_rng(seed)
    nh = rng.integers(16, 49, size=nsys)
    nzs = rng.integers(8, 25, size=nsys)
    ratio = 10.0 ** rng.uniform(2.0, 5.0, size=nsys)
    return [dict(nx=int(nh[i]), ny=int(nh[i]), nz=int(nzs[i]), ratio=float(ratio[i]),
                 field_seed=1000 * i + 500) for i in range(nsys)]


def batch_system(i: int, params=None) -> Problem:
    p = (params or batch_params())[i]
    kappa = lognormal_field((p["ny"], p["nx"], p["nz"]), seed=p["field_seed"])
    pr = slab_scalar(p["nx"], p["ny"], p["nz"], p["ratio"], kappa)
    pr.name = f"batch{i}"
    pr.leaf = 256
    pr.params.update(p)
    return pr


def batch_rhs(i: int, n: int, nrhs: int = 4) -> np.ndarray:
    """Column-major [n, nrhs] right-hand sides of system i (seed 1000*i + j)."""
    return np.stack([rhs(n, 1000 * i + j) for j in range(nrhs)], axis=1)


CONFIG_NAMES = ("laplace64", "slab64", "stokes128", "batch512", "stokes256")


def config(name: str) -> Problem:
    """The five named workloads.

    laplace64  2-D 5-point Laplacian, 64x64, Dirichlet; leaf 64, tol 1e-2.
    slab64     64x64x16 slab, ratio 1e4, log-normal kappa (seed 1); leaf 256.
    stokes128  128x128x20 two-component slab, ratio 1e4, kappa = 1; leaf 256.
    stokes256  256x256x32 two-component slab, ratio 1e4, log-normal; leaf 256.
    (batch512 is built system by system with ``batch_system``.)
    """
    if name == "laplace64":
        p = laplace2d(64)
        p.leaf, p.tol = 64, 1e-2
    elif name == "slab64":
        kap = lognormal_field((64, 64, 16), seed=1)
        p = slab_scalar(64, 64, 16, 1e4, kap)
        p.leaf, p.tol = 256, 1e-2
    elif name == "stokes128":
        p = slab_vector(128, 128, 20, 1e4)
        p.leaf, p.tol = 256, 1e-2
    elif name == "stokes256":
        kap = lognormal_field((256, 256, 32), seed=1)
        p = slab_vector(256, 256, 32, 1e4, kap)
        p.leaf, p.tol = 256, 1e-2
    else:
        raise ValueError(f"unknown config {name!r}")
    p.name = name
    return p


def config_variant(name: str, field_seed: int) -> Problem:
    """A named workload with another log-normal field seed: the same grid,
    pattern and parameters, other values (for steps whose values change)."""
    if name == "slab64":
        p = slab_scalar(64, 64, 16, 1e4, lognormal_field((64, 64, 16), seed=field_seed))
    elif name == "stokes256":
        p = slab_vector(256, 256, 32, 1e4, lognormal_field((256, 256, 32), seed=field_seed))
    elif name == "stokes128":
        p = slab_vector(128, 128, 20, 1e4, lognormal_field((128, 128, 20), seed=field_seed))
    elif name == "laplace64":
        p = laplace2d(64, eps=float(np.random.default_rng(field_seed).uniform(0.5, 2.0)))
    else:
        raise ValueError(f"unknown config {name!r}")
    base = config(name)
    p.leaf, p.tol, p.name = base.leaf, base.tol, f"{name}-field{field_seed}"
    return p

