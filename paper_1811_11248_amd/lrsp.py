"""ctypes binding of liblrsp.so (include/lrsp.h): argument marshalling only.

Every step of the factorization, the substitution sweeps and PCG runs in the
library's HIP kernels; this module only converts torch tensors and numpy
arrays to the pointers and sizes of the C interface.  PyTorch provides the
device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
import itertools
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
                ("val", C.c_void_p), ("h_rowptr", C.c_void_p), ("h_col", C.c_void_p),
                ("pattern_id", C.c_uint64)]


class Opts(C.Structure):
    _fields_ = [("tol_mode", C.c_int32), ("gemm_prec", C.c_int32), ("rank_mode", C.c_int32),
                ("exec_mode", C.c_int32), ("mlp_weights", C.c_void_p),
                ("autotune", C.c_int32), ("top_dense_threshold", C.c_int32), ("scheme", C.c_int32),
                ("reserved32b", C.c_int32), ("reserved", C.c_int64 * 4)]


class TreeView(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("nleaves", C.c_int32), ("n", C.c_int64),
                ("perm", C.POINTER(C.c_int64)), ("leaf_ptr", C.POINTER(C.c_int64))]


class Info(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("top_n", C.c_int32), ("top_clusters", C.c_int32),
                ("reserved", C.c_int32), ("flops", C.c_double * 6), ("bytes_factor", C.c_double),
                ("ms_levels", C.c_double), ("peak_bytes", C.c_int64), ("ms_analysis", C.c_double),
                ("levels_reused", C.c_int32), ("reserved2", C.c_int32),
                ("rank_bytes", C.c_double), ("rank_bytes_worst", C.c_double),
                ("rank_checks_passed", C.c_int32), ("rank_checks_failed", C.c_int32),
                ("rank_redo_levels", C.c_int32), ("rank_reruns", C.c_int32)]


class LevelView(C.Structure):
    _fields_ = [("nclusters", C.c_int32), ("ncolours", C.c_int32),
                ("sizes", C.POINTER(C.c_int32)), ("colour", C.POINTER(C.c_int32)),
                ("order", C.POINTER(C.c_int32)), ("ranks", C.POINTER(C.c_int32)),
                ("adj_ptr", C.POINTER(C.c_int32)), ("adj", C.POINTER(C.c_int32)),
                ("near", C.POINTER(C.c_int32)), ("far", C.POINTER(C.c_int32))]


class LevelStats(C.Structure):
    _fields_ = [("flops", C.c_double), ("sweep_bytes", C.c_double), ("factor_ms", C.c_double),
                ("solve_ms", C.c_double), ("applies", C.c_int64), ("dofs", C.c_int64), ("coarse", C.c_int64),
                ("nclusters", C.c_int32), ("reserved", C.c_int32), ("factor_bytes", C.c_int64),
                ("held_bytes", C.c_int64), ("work_bytes", C.c_int64), ("coarse_bytes", C.c_int64),
                ("panel_bytes", C.c_int64)]


class BatchInfo(C.Structure):
    _fields_ = [("nsys", C.c_int32), ("nlevels", C.c_int32), ("ntot", C.c_int64),
                ("flops", C.c_double * 6), ("ms_factor", C.c_double), ("ms_analysis", C.c_double),
                ("peak_bytes", C.c_int64), ("graph_factor", C.c_int32), ("graph_pcg", C.c_int32),
                ("coop_in_graph", C.c_int32), ("refactor_fallbacks", C.c_int32),
                ("tuned_levels", C.c_int32), ("graph_timeouts", C.c_int32),
                ("sched", C.c_int32 * 16), ("grid_cap", C.c_int32 * 16), ("tile", C.c_int32 * 16)]


class Timing(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


# (name, restype, argtypes) of every symbol declared in include/lrsp.h
SIGNATURES = [
    ("lrsp_tree_build", C.c_int, [C.POINTER(Grid), C.c_int32, C.POINTER(C.c_void_p)]),
    ("lrsp_tree_build_graph", C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_void_p)]),
    ("lrsp_tree_free", C.c_int, [C.c_void_p]),
    ("lrsp_tree_export", C.c_int, [C.c_void_p, C.POINTER(TreeView)]),
    ("lrsp_factor", C.c_int, [C.POINTER(CSR), C.c_void_p, C.c_double, C.POINTER(Opts), C.c_void_p,
                              C.POINTER(C.c_void_p)]),
    ("lrsp_factor_free", C.c_int, [C.c_void_p]),
    ("lrsp_apply", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    ("lrsp_pcg", C.c_int, [C.POINTER(CSR), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                           C.c_double, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                           C.c_void_p]),
    ("lrsp_pcg_noalloc", C.c_int, [C.POINTER(CSR), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                   C.c_double, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                   C.c_void_p]),
    ("lrsp_gmres", C.c_int, [C.POINTER(CSR), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                             C.c_double, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                             C.c_void_p]),
    ("lrsp_factor_info", C.c_int, [C.c_void_p, C.POINTER(Info)]),
    ("lrsp_factor_level", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(LevelView)]),
    ("lrsp_factor_level_stats", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(LevelStats)]),
    ("lrsp_factor_batched", C.c_int, [C.c_int32, C.POINTER(CSR), C.POINTER(C.c_void_p), C.c_double,
                                      C.POINTER(Opts), C.c_void_p, C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_int32)]),
    ("lrsp_refactor_batched", C.c_int, [C.c_void_p, C.POINTER(CSR), C.c_void_p, C.POINTER(C.c_int32)]),
    ("lrsp_batch_free", C.c_int, [C.c_void_p]),
    ("lrsp_apply_batched", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    ("lrsp_pcg_batched", C.c_int, [C.POINTER(CSR), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                   C.c_double, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double), C.c_void_p]),
    ("lrsp_batch_info_get", C.c_int, [C.c_void_p, C.POINTER(BatchInfo)]),
    ("lrsp_batch_level", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(LevelView)]),
    ("lrsp_batch_system_levels", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    ("lrsp_autotune_save", C.c_int, [C.c_char_p]),
    ("lrsp_autotune_load", C.c_int, [C.c_char_p]),
    ("lrsp_autotune_clear", C.c_int, []),
    ("lrsp_autotune_entries", C.c_int32, []),
    ("lrsp_mlp_nparams", C.c_int32, []),
    ("lrsp_mlp_init", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_uint64, C.c_void_p]),
    ("lrsp_mlp_loss_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    ("lrsp_mlp_train", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_float,
                                 C.c_void_p, C.c_void_p]),
    ("lrsp_mlp_predict", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    ("lrsp_factor_rank_features", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                            C.POINTER(C.c_float)]),
    ("lrsp_timing_enable", C.c_int, [C.c_int32]),
    ("lrsp_timing_reset", C.c_int, []),
    ("lrsp_timing_families", C.c_int, [C.c_uint32]),
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
        # torch first: its HIP runtime is then the one the library binds to
        # (loading the library first would bring a second runtime into the
        # process, and the two disagree about the devices)
        import torch  # noqa: F401
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

    @classmethod
    def from_graph(cls, adj_ptr, adj, nz: int, ncomp: int, leaf: int):
        """Extruded tree of an unstructured layer (lrsp_tree_build_graph)."""
        ap = np.ascontiguousarray(adj_ptr, dtype=np.int64)
        aj = np.ascontiguousarray(adj, dtype=np.int32)
        h = C.c_void_p()
        _check(lib().lrsp_tree_build_graph(int(ap.shape[0] - 1), ap.ctypes.data, aj.ctypes.data if aj.size else None,
                                           int(nz), int(ncomp), int(leaf), C.byref(h)))
        t = cls.__new__(cls)
        t.handle = h
        t.grid = (int(ap.shape[0] - 1), 1, int(nz), int(ncomp))
        t.leaf = leaf
        return t

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


_pattern_ids = itertools.count(1)


class DeviceMatrix:
    """CSR matrix resident in device memory (torch tensors) plus the host
    pattern.  The pattern arrays are private copies named by a pattern id of
    this process, so that a tree recognises them without comparing them."""

    def __init__(self, rowptr, col, val, device="cuda"):
        import torch
        self.h_rowptr = np.array(rowptr, dtype=np.int64, copy=True, order="C")
        self.h_col = np.array(col, dtype=np.int32, copy=True, order="C")
        self.pattern_id = next(_pattern_ids)
        self.rowptr = torch.from_numpy(self.h_rowptr).to(device)
        self.col = torch.from_numpy(self.h_col).to(device)
        self.h_rowptr.setflags(write=False)
        self.h_col.setflags(write=False)
        self.val = torch.as_tensor(np.asarray(val, dtype=np.float64)).to(device)
        self.n = int(self.h_rowptr.shape[0] - 1)
        self.nnz = int(self.h_col.shape[0])

    @classmethod
    def from_problem(cls, p, device="cuda"):
        return cls(p.rowptr, p.col, p.val, device)

    def csr(self) -> CSR:
        return CSR(self.n, self.nnz, self.rowptr.data_ptr(), self.col.data_ptr(),
                   self.val.data_ptr(), self.h_rowptr.ctypes.data, self.h_col.ctypes.data, self.pattern_id)


class Factor:
    """Hierarchical factor of a DeviceMatrix (lrsp_factor).

    mlp: parameters of the rank network (numpy float32 array or CPU/GPU
    tensor of lrsp_mlp_nparams() floats) to size the rank capacities from
    learned ranks (rank_mode 1)."""

    def __init__(self, A: DeviceMatrix, tree: Tree, tol: float, tol_mode="relative",
                 gemm_prec="f64", exec_mode="auto", stream=None, mlp=None, autotune=False,
                 top_dense=0, dc=True):
        o = Opts()
        o.scheme = 0 if dc else 1
        o.tol_mode = TOL_MODE[tol_mode]
        o.gemm_prec = PREC[gemm_prec]
        o.exec_mode = EXEC_MODE[exec_mode]
        o.autotune = 1 if autotune else 0
        o.top_dense_threshold = int(top_dense)
        self._mlp = None
        if mlp is not None:
            w = mlp.detach().cpu().numpy() if hasattr(mlp, "detach") else np.asarray(mlp)
            self._mlp = np.ascontiguousarray(w, dtype=np.float32)
            if self._mlp.size != mlp_nparams():
                raise ValueError("wrong number of MLP parameters")
            o.rank_mode = 1
            o.mlp_weights = self._mlp.ctypes.data
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
                "levels_reused": i.levels_reused, "peak_bytes": i.peak_bytes,
                "rank_bytes": i.rank_bytes, "rank_bytes_worst": i.rank_bytes_worst,
                "rank_checks_passed": i.rank_checks_passed, "rank_checks_failed": i.rank_checks_failed,
                "rank_redo_levels": i.rank_redo_levels, "rank_reruns": i.rank_reruns}

    def rank_features(self, lev: int):
        """(features [M, 12], predicted ranks [M]) of a level (rank_mode 1)."""
        M = self.level(lev)["nclusters"]
        f = np.zeros(M * 12)
        p = np.zeros(M, dtype=np.float32)
        _check(lib().lrsp_factor_rank_features(self.handle, int(lev), f.ctypes.data_as(C.POINTER(C.c_double)),
                                               p.ctypes.data_as(C.POINTER(C.c_float))))
        return f.reshape(M, 12), p

    def level(self, lev: int) -> dict:
        v = LevelView()
        _check(lib().lrsp_factor_level(self.handle, int(lev), C.byref(v)))
        return _level_dict(v)

    def level_stats(self, lev: int) -> dict:
        """Per-level flops, sweep bytes, sizes and (with timing on) GPU times;
        lev == info()['nlevels'] is the dense top."""
        r = LevelStats()
        _check(lib().lrsp_factor_level_stats(self.handle, int(lev), C.byref(r)))
        return {f: getattr(r, f) for f, _ in LevelStats._fields_ if f != "reserved"}

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lrsp_factor_free(self.handle)
            self.handle = None


def _level_dict(v: LevelView) -> dict:
    M = v.nclusters

    def arr(p, n):
        return np.ctypeslib.as_array(p, shape=(n,)).copy() if p and n else np.zeros(n, np.int32)
    ptr = arr(v.adj_ptr, M + 1)
    adj = arr(v.adj, int(ptr[-1])) if M else np.zeros(0, np.int32)
    out = {"nclusters": M, "ncolours": v.ncolours, "sizes": arr(v.sizes, M),
           "graph": [adj[ptr[c]:ptr[c + 1]].tolist() for c in range(M)]}
    if v.colour:
        out.update(colour=arr(v.colour, M), order=arr(v.order, M), ranks=arr(v.ranks, M))
    if v.near:
        out.update(near=arr(v.near, M), far=arr(v.far, M))
    return out


SCHED = {0: "persistent", 1: "per_colour", 2: "split"}


class Batch:
    """Batched factorization of several DeviceMatrix systems (lrsp_factor_batched).

    Vectors are packed: system i occupies rows off[i]:off[i+1] of each column.
    """

    def __init__(self, mats, trees, tol: float, tol_mode="relative", gemm_prec="f64",
                 exec_mode="auto", autotune=False, stream=None, raise_not_spd=True, top_dense=0):
        o = Opts()
        o.tol_mode = TOL_MODE[tol_mode]
        o.gemm_prec = PREC[gemm_prec]
        o.exec_mode = EXEC_MODE[exec_mode]
        o.autotune = 1 if autotune else 0
        o.top_dense_threshold = int(top_dense)
        self.mats = list(mats)
        self.trees = list(trees)
        n = len(self.mats)
        self._csrs = (CSR * n)(*[A.csr() for A in self.mats])
        th = (C.c_void_p * n)(*[t.handle.value for t in self.trees])
        h = C.c_void_p()
        status = (C.c_int32 * n)()
        st = lib().lrsp_factor_batched(n, self._csrs, th, float(tol), C.byref(o), _stream(stream),
                                       C.byref(h), status)
        self.handle = h if h.value else None
        self.status = np.array(status[:], dtype=np.int32)
        if st != ERR_NOT_SPD or raise_not_spd:
            _check(st)
        self.nsys = n
        self.sizes = np.array([A.n for A in self.mats], dtype=np.int64)
        self.off = np.concatenate([[0], np.cumsum(self.sizes)])

    def refactor(self, mats=None, stream=None):
        if mats is not None:
            self.mats = list(mats)
            self._csrs = (CSR * self.nsys)(*[A.csr() for A in self.mats])
        status = (C.c_int32 * self.nsys)()
        _check(lib().lrsp_refactor_batched(self.handle, self._csrs, _stream(stream), status))
        self.status = np.array(status[:], dtype=np.int32)

    def info(self) -> dict:
        i = BatchInfo()
        _check(lib().lrsp_batch_info_get(self.handle, C.byref(i)))
        nl = min(16, i.nlevels + 1)
        return {"nsys": i.nsys, "nlevels": i.nlevels, "ntot": i.ntot,
                "flops": dict(zip(("potrf", "trsm", "cpqr", "applyq", "schur", "top"), i.flops)),
                "ms_factor": i.ms_factor, "ms_analysis": i.ms_analysis, "peak_bytes": i.peak_bytes,
                "graph_factor": i.graph_factor, "graph_pcg": i.graph_pcg,
                "refactor_fallbacks": i.refactor_fallbacks, "tuned_levels": i.tuned_levels,
                "graph_timeouts": i.graph_timeouts,
                "sched": [SCHED.get(i.sched[l], "?") for l in range(nl)],
                "grid_cap": list(i.grid_cap[:nl]),
                "tile": [32 if i.tile[l] == 0 else 16 for l in range(nl)]}

    def system_levels(self, sys: int) -> int:
        n = C.c_int32()
        _check(lib().lrsp_batch_system_levels(self.handle, int(sys), C.byref(n)))
        return int(n.value)

    def level(self, sys: int, lev: int) -> dict:
        v = LevelView()
        _check(lib().lrsp_batch_level(self.handle, int(sys), int(lev), C.byref(v)))
        return _level_dict(v)

    def pack(self, vecs, device="cuda"):
        """Packs per-system arrays ([n_i] or [n_i, nrhs]) into a device [ntot, nrhs] tensor."""
        import torch
        cols = [torch.as_tensor(np.asarray(v, dtype=np.float64)).reshape(len(v), -1) for v in vecs]
        return torch.cat(cols, 0).to(device)

    def unpack(self, X):
        return [X[self.off[i]:self.off[i + 1]] for i in range(self.nsys)]

    def apply(self, B, stream=None):
        """x = M^{-1} b for a packed device tensor [ntot] or [ntot, nrhs]."""
        import torch
        nrhs = 1 if B.dim() == 1 else B.shape[1]
        bb = B if B.dim() == 1 else B.t().contiguous()
        out = torch.empty_like(bb)
        _check(lib().lrsp_apply_batched(self.handle, bb.data_ptr(), out.data_ptr(), nrhs, _stream(stream)))
        return out if B.dim() == 1 else out.view(nrhs, -1).t()

    def pcg(self, B, rtol=1e-8, maxit=1000, stream=None, raise_no_conv=True, x=None):
        """PCG on every (system, column); returns (X, iters[nrhs, nsys], relres[nrhs, nsys])."""
        import torch
        nrhs = 1 if B.dim() == 1 else B.shape[1]
        bb = B if B.dim() == 1 else B.t().contiguous()
        xx = torch.empty_like(bb) if x is None else x
        np_ = nrhs * self.nsys
        it = (C.c_int32 * np_)()
        rr = (C.c_double * np_)()
        st = lib().lrsp_pcg_batched(self._csrs, self.handle, bb.data_ptr(), xx.data_ptr(), nrhs,
                                    float(rtol), int(maxit), it, rr, _stream(stream))
        if st != ERR_NO_CONV or raise_no_conv:
            _check(st)
        X = xx if B.dim() == 1 else xx.view(nrhs, -1).t()
        return (X, np.array(it[:], dtype=np.int64).reshape(nrhs, self.nsys),
                np.array(rr[:]).reshape(nrhs, self.nsys))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lrsp_batch_free(self.handle)
            self.handle = None


def mlp_nparams() -> int:
    return int(lib().lrsp_mlp_nparams())


def mlp_init(X, t, seed=1, stream=None):
    """New parameter tensor (device, fp32) initialised from data X [n, 12], t [n]."""
    import torch
    P = torch.zeros(mlp_nparams(), dtype=torch.float32, device=X.device)
    _check(lib().lrsp_mlp_init(P.data_ptr(), X.data_ptr(), t.data_ptr(), int(X.shape[0]), int(seed),
                               _stream(stream)))
    return P


def mlp_loss_grad(P, X, t, stream=None):
    import torch
    g = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device=P.device)
    _check(lib().lrsp_mlp_loss_grad(P.data_ptr(), X.data_ptr(), t.data_ptr(), int(X.shape[0]),
                                    g.data_ptr(), loss.data_ptr(), _stream(stream)))
    return float(loss.item()), g


def mlp_train(P, X, t, steps, lr=1e-2, stream=None):
    """Trains P in place; returns the loss before every step (device tensor)."""
    import torch
    trace = torch.empty(max(1, steps), dtype=torch.float32, device=P.device)
    _check(lib().lrsp_mlp_train(P.data_ptr(), X.data_ptr(), t.data_ptr(), int(X.shape[0]), int(steps),
                                float(lr), trace.data_ptr(), _stream(stream)))
    return trace[:steps]


def mlp_predict(P, X, stream=None):
    import torch
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(lib().lrsp_mlp_predict(P.data_ptr(), X.data_ptr(), int(X.shape[0]), y.data_ptr(),
                                  _stream(stream)))
    return y


def autotune_save(path: str):
    _check(lib().lrsp_autotune_save(path.encode()))


def autotune_load(path: str):
    _check(lib().lrsp_autotune_load(path.encode()))


def autotune_clear():
    _check(lib().lrsp_autotune_clear())


def autotune_entries() -> int:
    return int(lib().lrsp_autotune_entries())


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


PCG_NOALLOC_MAX_N = 1048576


def pcg(A: DeviceMatrix, F: Factor, b, rtol=1e-8, maxit=1000, stream=None, raise_no_conv=True,
        noalloc=False, x=None):
    """PCG with the factor; returns (x, iters, relres) with per-column numpy arrays.

    noalloc: call lrsp_pcg_noalloc (work vectors in the library's static
    device array, n <= PCG_NOALLOC_MAX_N); x: optional output tensor of the
    layout of b (for b of shape [n, nrhs], its transpose made contiguous)."""
    import torch
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    bb = b if b.dim() == 1 else b.t().contiguous()
    x = torch.empty_like(bb) if x is None else x
    it = (C.c_int32 * nrhs)()
    rr = (C.c_double * nrhs)()
    csr = A.csr()
    fn = lib().lrsp_pcg_noalloc if noalloc else lib().lrsp_pcg
    st = fn(C.byref(csr), F.handle, bb.data_ptr(), x.data_ptr(), nrhs, float(rtol),
            int(maxit), it, rr, _stream(stream))
    if st != ERR_NO_CONV or raise_no_conv:
        _check(st)
    xo = x if b.dim() == 1 else x.view(nrhs, -1).t()
    return xo, np.array(it[:], dtype=np.int64), np.array(rr[:])


def gmres(A: DeviceMatrix, F: Factor, b, rtol=1e-12, restart=200, maxit=1000, stream=None,
          raise_no_conv=True):
    """Right-preconditioned restarted GMRES with the factor; returns
    (x, iters, relres) with per-column numpy arrays."""
    import torch
    nrhs = 1 if b.dim() == 1 else b.shape[1]
    bb = b if b.dim() == 1 else b.t().contiguous()
    x = torch.empty_like(bb)
    it = (C.c_int32 * nrhs)()
    rr = (C.c_double * nrhs)()
    csr = A.csr()
    st = lib().lrsp_gmres(C.byref(csr), F.handle, bb.data_ptr(), x.data_ptr(), nrhs, int(restart),
                          float(rtol), int(maxit), it, rr, _stream(stream))
    if st != ERR_NO_CONV or raise_no_conv:
        _check(st)
    xo = x if b.dim() == 1 else x.view(nrhs, -1).t()
    return xo, np.array(it[:], dtype=np.int64), np.array(rr[:])


TIMING_FAMILIES = {"eliminate": 0, "forward": 1, "backward": 2, "split_gather": 3,
                   "split_potrf": 4, "split_trsm": 5, "split_cpqr": 6, "split_applyq": 7,
                   "split_schur": 8, "split_writeback": 9, "fused": 10, "spmv": 11}


def timing_enable(on: bool = True):
    _check(lib().lrsp_timing_enable(1 if on else 0))


def timing_families(names=None):
    """Restrict event recording to the named families (None: all)."""
    mask = 0xFFFFFFFF if names is None else sum(1 << TIMING_FAMILIES[n] for n in names)
    _check(lib().lrsp_timing_families(mask))


def timing_reset():
    _check(lib().lrsp_timing_reset())


def timing_read(family: str) -> dict:
    t = Timing()
    _check(lib().lrsp_timing_read(TIMING_FAMILIES[family], C.byref(t)))
    return {"launches": int(t.launches), "total_ms": t.total_ms, "flops": t.flops, "bytes": t.bytes}
