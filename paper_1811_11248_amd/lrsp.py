"""ctypes binding of liblrsp.so (include/lrsp.h): argument marshalling only.

Every step of the factorization, the substitution sweeps and PCG runs in the
library's HIP kernels; this module only converts torch tensors and numpy
arrays to the pointers and sizes of the C interface.  PyTorch provides the
device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrsp.so")

OK, ERR_ARG, ERR_NOT_SPD, ERR_HIP, ERR_OOM, ERR_NO_CONV, ERR_INTERNAL = range(7)
PREC = {"f64": 0, "f32": 1, "bf16": 2}
TOL_MODE = {"relative": 0, "absolute": 1}
EXEC_MODE = {"auto": 0, "colour": 1, "level": 2, "split": 3}


class LrspError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lrsp error {status}: {msg}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("ncomp", C.c_int32)]


class CSR(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("h_rowptr", C.c_void_p), ("h_col", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("tol_mode", C.c_int32), ("gemm_prec", C.c_int32), ("rank_mode", C.c_int32),
                ("exec_mode", C.c_int32), ("mlp_weights", C.c_void_p),
                ("reserved", C.c_int64 * 6)]


class TreeView(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("nleaves", C.c_int32), ("n", C.c_int64),
                ("perm", C.POINTER(C.c_int64)), ("leaf_ptr", C.POINTER(C.c_int64))]


class Info(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("top_n", C.c_int32), ("top_clusters", C.c_int32),
                ("reserved", C.c_int32), ("flops", C.c_double * 6), ("bytes_factor", C.c_double),
                ("ms_levels", C.c_double), ("peak_bytes", C.c_int64), ("ms_analysis", C.c_double),
                ("levels_reused", C.c_int32), ("reserved2", C.c_int32)]


class LevelView(C.Structure):
    _fields_ = [("nclusters", C.c_int32), ("ncolours", C.c_int32),
                ("sizes", C.POINTER(C.c_int32)), ("colour", C.POINTER(C.c_int32)),
                ("order", C.POINTER(C.c_int32)), ("ranks", C.POINTER(C.c_int32)),
                ("adj_ptr", C.POINTER(C.c_int32)), ("adj", C.POINTER(C.c_int32))]


class Timing(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


# (name, restype, argtypes) of every symbol declared in include/lrsp.h
SIGNATURES = [
    ("lrsp_tree_build", C.c_int, [C.POINTER(Grid), C.c_int32, C.POINTER(C.c_void_p)]),
    ("lrsp_tree_free", C.c_int, [C.c_void_p]),
    ("lrsp_tree_export", C.c_int, [C.c_void_p, C.POINTER(TreeView)]),
    ("lrsp_factor", C.c_int, [C.POINTER(CSR), C.c_void_p, C.c_double, C.POINTER(Opts), C.c_void_p,
                              C.POINTER(C.c_void_p)]),
    ("lrsp_factor_free", C.c_int, [C.c_void_p]),
    ("lrsp_apply", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    ("lrsp_pcg", C.c_int, [C.POINTER(CSR), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                           C.c_double, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                           C.c_void_p]),
    ("lrsp_factor_info", C.c_int, [C.c_void_p, C.POINTER(Info)]),
    ("lrsp_factor_level", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(LevelView)]),
    ("lrsp_timing_enable", C.c_int, [C.c_int32]),
    ("lrsp_timing_reset", C.c_int, []),
    ("lrsp_timing_read", C.c_int, [C.c_int32, C.POINTER(Timing)]),
    ("lrsp_last_error_info", C.c_char_p, []),
    ("lrsp_status_str", C.c_char_p, [C.c_int]),
]

_lib = None


def lib():
    """Loads liblrsp.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1811_11248_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _check(st: int):
    if st != OK:
        msg = lib().lrsp_last_error_info().decode() or lib().lrsp_status_str(st).decode()
        raise LrspError(st, msg)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Tree:
    """Cluster tree of an extruded grid (lrsp_tree_build)."""

    def __init__(self, grid, leaf: int):
        g = Grid(*[int(v) for v in grid])
        h = C.c_void_p()
        _check(lib().lrsp_tree_build(C.byref(g), int(leaf), C.byref(h)))
        self.handle = h
        self.grid = tuple(grid)
        self.leaf = leaf

    def export(self):
        v = TreeView()
        _check(lib().lrsp_tree_export(self.handle, C.byref(v)))
        perm = np.ctypeslib.as_array(v.perm, shape=(v.n,)).copy()
        ptr = np.ctypeslib.as_array(v.leaf_ptr, shape=(v.nleaves + 1,)).copy()
        return {"nlevels": v.nlevels, "perm": perm, "leaf_ptr": ptr,
                "leaf_dofs": [perm[ptr[c]:ptr[c + 1]] for c in range(v.nleaves)]}

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lrsp_tree_free(self.handle)
            self.handle = None


class DeviceMatrix:
    """CSR matrix resident in device memory (torch tensors) plus the host pattern."""

    def __init__(self, rowptr, col, val, device="cuda"):
        import torch
        self.h_rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.h_col = np.ascontiguousarray(col, dtype=np.int32)
        self.rowptr = torch.from_numpy(self.h_rowptr).to(device)
        self.col = torch.from_numpy(self.h_col).to(device)
        self.val = torch.as_tensor(np.asarray(val, dtype=np.float64)).to(device)
        self.n = int(self.h_rowptr.shape[0] - 1)
        self.nnz = int(self.h_col.shape[0])

    @classmethod
    def from_problem(cls, p, device="cuda"):
        return cls(p.rowptr, p.col, p.val, device)

    def csr(self) -> CSR:
        return CSR(self.n, self.nnz, self.rowptr.data_ptr(), self.col.data_ptr(),
                   self.val.data_ptr(), self.h_rowptr.ctypes.data, self.h_col.ctypes.data)


class Factor:
    """Hierarchical factor of a DeviceMatrix (lrsp_factor)."""

    def __init__(self, A: DeviceMatrix, tree: Tree, tol: float, tol_mode="relative",
                 gemm_prec="f64", exec_mode="auto", stream=None):
        o = Opts()
        o.tol_mode = TOL_MODE[tol_mode]
        o.gemm_prec = PREC[gemm_prec]
        o.exec_mode = EXEC_MODE[exec_mode]
        h = C.c_void_p()
        self._csr = A.csr()
        self.A = A
        self.tree = tree
        _check(lib().lrsp_factor(C.byref(self._csr), tree.handle, float(tol), C.byref(o),
                                 _stream(stream), C.byref(h)))
        self.handle = h

    def info(self) -> dict:
        i = Info()
        _check(lib().lrsp_factor_info(self.handle, C.byref(i)))
        return {"nlevels": i.nlevels, "top_n": i.top_n, "top_clusters": i.top_clusters,
                "flops": dict(zip(("potrf", "trsm", "cpqr", "applyq", "schur", "top"), i.flops)),
                "bytes_factor": i.bytes_factor, "ms": i.ms_levels, "ms_analysis": i.ms_analysis,
                "levels_reused": i.levels_reused}

    def level(self, lev: int) -> dict:
        v = LevelView()
        _check(lib().lrsp_factor_level(self.handle, int(lev), C.byref(v)))
        M = v.nclusters

        def arr(p, n):
            return np.ctypeslib.as_array(p, shape=(n,)).copy() if p and n else np.zeros(n, np.int32)
        ptr = arr(v.adj_ptr, M + 1)
        adj = arr(v.adj, int(ptr[-1])) if M else np.zeros(0, np.int32)
        out = {"nclusters": M, "ncolours": v.ncolours, "sizes": arr(v.sizes, M),
               "graph": [adj[ptr[c]:ptr[c + 1]].tolist() for c in range(M)]}
        if v.colour:
            out.update(colour=arr(v.colour, M), order=arr(v.order, M), ranks=arr(v.ranks, M))
        return out

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lrsp_factor_free(self.handle)
            self.handle = None


def tree_build(grid, leaf):
    return Tree(grid, leaf)


def factor(A: DeviceMatrix, tree: Tree, tol: float, **kw) -> Factor:
    return Factor(A, tree, tol, **kw)


def apply(F: Factor, b, x=None, stream=None):
    """x = M^{-1} b for device tensors of shape [n] or [n, nrhs] (column-major)."""
    import torch
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    bb = b if b.dim() == 1 else b.t().contiguous()
    out = torch.empty_like(bb) if x is None else x
    _check(lib().lrsp_apply(F.handle, bb.data_ptr(), out.data_ptr(), nrhs, _stream(stream)))
    return out if b.dim() == 1 else out.view(nrhs, -1).t()


def pcg(A: DeviceMatrix, F: Factor, b, rtol=1e-8, maxit=1000, stream=None, raise_no_conv=True):
    """PCG with the factor; returns (x, iters, relres) with per-column numpy arrays."""
    import torch
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    bb = b if b.dim() == 1 else b.t().contiguous()
    x = torch.empty_like(bb)
    it = (C.c_int32 * nrhs)()
    rr = (C.c_double * nrhs)()
    csr = A.csr()
    st = lib().lrsp_pcg(C.byref(csr), F.handle, bb.data_ptr(), x.data_ptr(), nrhs, float(rtol),
                        int(maxit), it, rr, _stream(stream))
    if st != ERR_NO_CONV or raise_no_conv:
        _check(st)
    xo = x if b.dim() == 1 else x.view(nrhs, -1).t()
    return xo, np.array(it[:], dtype=np.int64), np.array(rr[:])


TIMING_FAMILIES = {"eliminate": 0, "forward": 1, "backward": 2, "split_gather": 3,
                   "split_potrf": 4, "split_trsm": 5, "split_cpqr": 6, "split_applyq": 7,
                   "split_schur": 8, "split_writeback": 9, "fused": 10}


def timing_enable(on: bool = True):
    _check(lib().lrsp_timing_enable(1 if on else 0))


def timing_reset():
    _check(lib().lrsp_timing_reset())


def timing_read(family: str) -> dict:
    t = Timing()
    _check(lib().lrsp_timing_read(TIMING_FAMILIES[family], C.byref(t)))
    return {"launches": int(t.launches), "total_ms": t.total_ms, "flops": t.flops, "bytes": t.bytes}
