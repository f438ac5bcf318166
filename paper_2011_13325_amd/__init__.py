"""Python binding of libeamg, the MI355X edge-matrix AMG-PCG library (C ABI in include/eamg.h).

Argument marshalling only: every step of setup and solve runs in the library (host C++ setup,
HIP kernels on the GPU).  Device buffers are torch tensors on a HIP device; host inputs are
numpy arrays.  Importing works without a GPU (so the ABI can be checked); the library must be
built (``python -m paper_2011_13325_amd.build``) or loading fails loudly.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeamg.so")

EAMG_OK = 0
EAMG_NOT_CONVERGED = 1
EAMG_ERR_INVALID_ARG = -1
EAMG_ERR_UNSUPPORTED_KERNEL = -2
EAMG_ERR_NOT_SPD = -3
EAMG_ERR_BREAKDOWN = -4
EAMG_ERR_HIP = -5
EAMG_ERR_OOM = -6

EAMG_PRECOND_NONE = 0
EAMG_PRECOND_VCYCLE = 1
EAMG_PRECOND_VCYCLE_FP32 = 2

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "INVALID_ARG", -2: "UNSUPPORTED_KERNEL",
                -3: "NOT_SPD", -4: "BREAKDOWN", -5: "HIP", -6: "OOM"}

# Every symbol include/eamg.h declares.
EXPORTED = ["eamg_default_setup_params", "eamg_default_solve_params", "eamg_setup", "eamg_solve",
            "eamg_vcycle", "eamg_stats", "eamg_level_info_get", "eamg_export_level",
            "eamg_traffic_model", "eamg_destroy", "eamg_last_error", "eamg_host_match",
            "eamg_criteria_eval",
            "eamg_profile_enable", "eamg_profile_read", "eamg_solve_batch", "eamg_solve_multi",
            "eamg_autotune", "eamg_gnn_create", "eamg_gnn_params", "eamg_gnn_forward",
            "eamg_gnn_loss_grad", "eamg_gnn_train", "eamg_gnn_destroy", "eamg_coarsening_stats",
            "eamg_gnn_samples", "eamg_dense_tail", "eamg_solve_coefficients", "eamg_setup_phases",
            "eamg_vcycle_noalloc", "eamg_fuse", "eamg_solve_fused"]


class eamg_problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_vertices", ctypes.c_int32),
                ("coords", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("vals", ctypes.c_void_p),
                ("dirichlet", ctypes.c_void_p), ("kernel", ctypes.c_void_p),
                ("k_kernel", ctypes.c_int32), ("edges", ctypes.c_void_p),
                ("n_edges", ctypes.c_int64)]


class eamg_setup_params(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("delta", ctypes.c_int32), ("R", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("coarsest_max_dofs", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("omega", ctypes.c_double),
                ("cap_aux", ctypes.c_int32), ("cap_std_l0", ctypes.c_int32),
                ("cap_std", ctypes.c_int32), ("pinv_rtol", ctypes.c_double),
                ("tie_rtol", ctypes.c_double), ("vcycle_fp32", ctypes.c_int32),
                ("gnn", ctypes.c_void_p), ("gnn_skip", ctypes.c_double),
                ("gnn_record", ctypes.c_int32), ("mu_s_only", ctypes.c_int32),
                ("gpu_criteria", ctypes.c_int32), ("dense_tail_dofs", ctypes.c_int32),
                ("dense_tail_fp32", ctypes.c_int32)]


class eamg_solve_params(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_it", ctypes.c_int32),
                ("use_x0", ctypes.c_int32), ("precond", ctypes.c_int32)]


class eamg_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("ms", ctypes.c_double),
                ("status", ctypes.c_int32)]


class eamg_level_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("bs", ctypes.c_int32), ("nnzb_A", ctypes.c_int64),
                ("n_coarse", ctypes.c_int32), ("k_coarse", ctypes.c_int32),
                ("nnzb_P", ctypes.c_int64), ("n_colors", ctypes.c_int32)]


class eamg_setup_phase(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("seconds", ctypes.c_double), ("where", ctypes.c_int32)]


class eamg_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


_lib = None


def lib():
    """The loaded libeamg (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: the HIP library has not been built "
                           "(python -m paper_2011_13325_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.eamg_default_setup_params.argtypes = [P(eamg_setup_params)]
    L.eamg_default_setup_params.restype = None
    L.eamg_default_solve_params.argtypes = [P(eamg_solve_params)]
    L.eamg_default_solve_params.restype = None
    L.eamg_setup.argtypes = [P(eamg_problem), P(eamg_setup_params), vp, P(vp)]
    L.eamg_setup.restype = ctypes.c_int
    L.eamg_solve.argtypes = [vp, vp, vp, P(eamg_solve_params), vp, P(eamg_solve_info)]
    L.eamg_solve.restype = ctypes.c_int
    L.eamg_solve_batch.argtypes = [vp, i32, vp, i64, vp, P(eamg_solve_params), vp, P(eamg_solve_info)]
    L.eamg_solve_batch.restype = ctypes.c_int
    fp = P(ctypes.c_float)
    L.eamg_gnn_create.argtypes = [vp, ctypes.c_uint64, P(vp)]
    L.eamg_gnn_create.restype = ctypes.c_int
    L.eamg_gnn_params.argtypes = [vp, vp]
    L.eamg_gnn_params.restype = ctypes.c_int
    L.eamg_gnn_forward.argtypes = [vp, i64, i32, vp, vp, vp]
    L.eamg_gnn_forward.restype = ctypes.c_int
    L.eamg_gnn_loss_grad.argtypes = [vp, i64, i32, vp, vp, vp, vp, P(dp), vp]
    L.eamg_gnn_loss_grad.restype = ctypes.c_int
    L.eamg_gnn_train.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, i32, ctypes.c_float, vp]
    L.eamg_gnn_train.restype = ctypes.c_int
    L.eamg_gnn_destroy.argtypes = [vp]
    L.eamg_gnn_destroy.restype = None
    L.eamg_coarsening_stats.argtypes = [vp, P(i64), P(i64), P(i64), P(i32)]
    L.eamg_coarsening_stats.restype = ctypes.c_int
    L.eamg_gnn_samples.argtypes = [vp, i32, P(i64), P(i32), vp, vp, vp, vp]
    L.eamg_gnn_samples.restype = ctypes.c_int
    L.eamg_autotune.argtypes = [vp, i32, vp, P(dp), P(dp)]
    L.eamg_autotune.restype = ctypes.c_int
    L.eamg_solve_multi.argtypes = [i32, P(vp), P(vp), P(vp), P(eamg_solve_params), vp, P(eamg_solve_info)]
    L.eamg_solve_multi.restype = ctypes.c_int
    L.eamg_fuse.argtypes = [i32, P(vp), i32, vp, P(vp)]
    L.eamg_fuse.restype = ctypes.c_int
    L.eamg_solve_fused.argtypes = [vp, P(vp), P(vp), P(eamg_solve_params), vp, P(eamg_solve_info)]
    L.eamg_solve_fused.restype = ctypes.c_int
    L.eamg_vcycle.argtypes = [vp, vp, vp, i32, vp]
    L.eamg_vcycle.restype = ctypes.c_int
    L.eamg_vcycle_noalloc.argtypes = [vp, vp, vp, i32, vp]
    L.eamg_vcycle_noalloc.restype = ctypes.c_int
    L.eamg_stats.argtypes = [vp, P(i32), vp, vp, P(dp), P(dp)]
    L.eamg_stats.restype = ctypes.c_int
    L.eamg_level_info_get.argtypes = [vp, i32, P(eamg_level_info)]
    L.eamg_level_info_get.restype = ctypes.c_int
    L.eamg_export_level.argtypes = [vp, i32] + [vp] * 8
    L.eamg_export_level.restype = ctypes.c_int
    L.eamg_traffic_model.argtypes = [vp, i32, P(dp), P(dp)]
    L.eamg_traffic_model.restype = ctypes.c_int
    L.eamg_destroy.argtypes = [vp]
    L.eamg_destroy.restype = None
    L.eamg_last_error.argtypes = []
    L.eamg_last_error.restype = ctypes.c_char_p
    L.eamg_host_match.argtypes = [i32, i32, vp, i64, vp, vp, vp, vp, P(eamg_setup_params), vp,
                                  P(i32), vp, P(dp)]
    L.eamg_host_match.restype = ctypes.c_int
    L.eamg_criteria_eval.argtypes = [i32, i32, vp, i64, vp, vp, vp, i64, vp, i64, vp, dp, i32, vp,
                                     vp, vp]
    L.eamg_criteria_eval.restype = ctypes.c_int
    L.eamg_profile_enable.argtypes = [vp, i32]
    L.eamg_profile_enable.restype = ctypes.c_int
    L.eamg_profile_read.argtypes = [vp, i32, P(eamg_kernel_stat), P(i32)]
    L.eamg_profile_read.restype = ctypes.c_int
    L.eamg_setup_phases.argtypes = [vp, i32, P(eamg_setup_phase), P(i32)]
    L.eamg_setup_phases.restype = ctypes.c_int
    L.eamg_dense_tail.argtypes = [vp, P(i32), P(i32)]
    L.eamg_dense_tail.restype = ctypes.c_int
    L.eamg_solve_coefficients.argtypes = [vp, i32, vp, vp, P(i32)]
    L.eamg_solve_coefficients.restype = ctypes.c_int
    _lib = L
    return L


class EamgError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib().eamg_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def eamg_default_setup_params(**overrides) -> eamg_setup_params:
    p = eamg_setup_params()
    lib().eamg_default_setup_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def eamg_last_error() -> str:
    return lib().eamg_last_error().decode()


def _problem(dim, coords, row_ptr, col_idx, vals, dirichlet=None, kernel=None, edges=None):
    keep = {
        "coords": np.ascontiguousarray(coords, dtype=np.float64),
        "row_ptr": np.ascontiguousarray(row_ptr, dtype=np.int32),
        "col_idx": np.ascontiguousarray(col_idx, dtype=np.int32),
        "vals": np.ascontiguousarray(vals, dtype=np.float64),
        "dirichlet": None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8),
        "kernel": None if kernel is None else np.asfortranarray(kernel, dtype=np.float64),
        "edges": None if edges is None else np.ascontiguousarray(edges, dtype=np.int32),
    }
    pb = eamg_problem()
    pb.dim = dim
    pb.n_vertices = keep["coords"].shape[0]
    pb.coords = _ptr(keep["coords"])
    pb.row_ptr = _ptr(keep["row_ptr"])
    pb.col_idx = _ptr(keep["col_idx"])
    pb.vals = _ptr(keep["vals"])
    pb.dirichlet = _ptr(keep["dirichlet"])
    pb.kernel = _ptr(keep["kernel"])
    pb.k_kernel = 6 if dim == 3 else 1
    pb.edges = _ptr(keep["edges"])
    pb.n_edges = 0 if edges is None else keep["edges"].shape[0]
    return pb, keep


def eamg_setup(dim, coords, row_ptr, col_idx, vals, dirichlet=None, params=None, stream=None,
               kernel=None, edges=None):
    """Returns an opaque handle (ctypes.c_void_p).  Raises EamgError on failure."""
    pb, keep = _problem(dim, coords, row_ptr, col_idx, vals, dirichlet, kernel, edges)
    h = ctypes.c_void_p()
    st = lib().eamg_setup(ctypes.byref(pb), ctypes.byref(params) if params is not None else None,
                          _stream(stream), ctypes.byref(h))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_setup")
    return h


def eamg_solve(h, b, x, rtol=1e-8, max_it=1000, use_x0=False, precond=True, stream=None):
    """b, x: float64 device tensors of n*dim entries.  Returns (status, info dict)."""
    sp = eamg_solve_params(rtol, max_it, int(use_x0), int(precond))
    info = eamg_solve_info()
    st = lib().eamg_solve(h, _dptr(b), _dptr(x), ctypes.byref(sp), _stream(stream),
                          ctypes.byref(info))
    if st < 0:
        raise EamgError(st, "eamg_solve")
    return st, dict(iterations=info.iterations, rel_res=info.rel_res,
                    rel_res_true=info.rel_res_true, ms=info.ms)


def eamg_solve_batch(h, B, X, rtol=1e-8, max_it=1000, use_x0=False, precond=True, stream=None):
    """B, X: float64 device tensors of shape (nrhs, n*dim), rows contiguous (column c of the
    batch is row c).  Returns (status, [info dict per right-hand side])."""
    nrhs, ndof = B.shape
    assert X.shape == B.shape and B.stride(1) == 1 and X.stride(1) == 1 and B.stride(0) == X.stride(0)
    sp = eamg_solve_params(rtol, max_it, int(use_x0), int(precond))
    infos = (eamg_solve_info * nrhs)()
    st = lib().eamg_solve_batch(h, nrhs, _dptr(B), B.stride(0), _dptr(X), ctypes.byref(sp),
                                _stream(stream), infos)
    if st < 0:
        raise EamgError(st, "eamg_solve_batch")
    return st, [dict(iterations=i.iterations, rel_res=i.rel_res, rel_res_true=i.rel_res_true,
                     ms=i.ms, status=i.status) for i in infos]


def eamg_solve_multi(hs, bs, xs, rtol=1e-8, max_it=1000, use_x0=False, precond=True, stream=None):
    """hs: hierarchy handles; bs, xs: float64 device tensors, one per system.
    Returns (status, [info dict per system])."""
    n = len(hs)
    assert len(bs) == n and len(xs) == n
    H = (ctypes.c_void_p * n)(*[ctypes.c_void_p(h) if not isinstance(h, ctypes.c_void_p) else h for h in hs])
    Bp = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
    Xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    sp = eamg_solve_params(rtol, max_it, int(use_x0), int(precond))
    infos = (eamg_solve_info * n)()
    st = lib().eamg_solve_multi(n, H, Bp, Xp, ctypes.byref(sp), _stream(stream), infos)
    if st < 0:
        raise EamgError(st, "eamg_solve_multi")
    return st, [dict(iterations=i.iterations, rel_res=i.rel_res, rel_res_true=i.rel_res_true,
                     ms=i.ms, status=i.status) for i in infos]


def eamg_fuse(hs, dense_tail_dofs=0, stream=None):
    """Fused hierarchy handle of the hierarchy handles hs (eamg_destroy frees it)."""
    n = len(hs)
    H = (ctypes.c_void_p * n)(*[ctypes.c_void_p(h) if not isinstance(h, ctypes.c_void_p) else h for h in hs])
    out = ctypes.c_void_p()
    st = lib().eamg_fuse(n, H, int(dense_tail_dofs), _stream(stream), ctypes.byref(out))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_fuse")
    return out.value


def eamg_solve_fused(hf, bs, xs, rtol=1e-8, max_it=1000, use_x0=False, precond=True, stream=None):
    """hf: fused hierarchy handle; bs, xs: float64 device tensors, one per system.
    Returns (status, [info dict per system])."""
    n = len(bs)
    assert len(xs) == n
    Bp = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bs])
    Xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    sp = eamg_solve_params(rtol, max_it, int(use_x0), int(precond))
    infos = (eamg_solve_info * n)()
    st = lib().eamg_solve_fused(hf, Bp, Xp, ctypes.byref(sp), _stream(stream), infos)
    if st < 0:
        raise EamgError(st, "eamg_solve_fused")
    return st, [dict(iterations=i.iterations, rel_res=i.rel_res, rel_res_true=i.rel_res_true,
                     ms=i.ms, status=i.status) for i in infos]


GNN_FEATURES = 12
GNN_PARAMS = 9153


# Owning wrappers still open.  They are closed at interpreter exit by an atexit hook, which runs
# before the C-level exit handlers (the HIP runtime's and a profiler tool's): freeing device
# objects from __del__ during the interpreter's final collection could otherwise reach a
# runtime or tool that has already shut down.
_OPEN = weakref.WeakSet()


@atexit.register
def close_all():
    """Close every Hierarchy, Fused and EdgeNet that is still open."""
    for obj in list(_OPEN):
        try:
            obj.close()
        except Exception:
            pass


class EdgeNet:
    """The edge-scoring network (eamg_gnn_*): parameters on the device, host arrays in/out."""

    def __init__(self, params=None, seed=0):
        h = ctypes.c_void_p()
        pp = None
        if params is not None:
            self._p = np.ascontiguousarray(params, dtype=np.float32)
            assert self._p.size == GNN_PARAMS
            pp = _ptr(self._p)
        st = lib().eamg_gnn_create(pp, int(seed), ctypes.byref(h))
        if st != EAMG_OK:
            raise EamgError(st, "eamg_gnn_create")
        self.h = h
        _OPEN.add(self)

    @staticmethod
    def _graph(X, edges):
        X = np.ascontiguousarray(X, dtype=np.float32)
        edges = np.ascontiguousarray(edges, dtype=np.int32)
        assert X.ndim == 2 and X.shape[1] == GNN_FEATURES and edges.shape == (X.shape[0], 2)
        return X, edges

    def params(self):
        out = np.zeros(GNN_PARAMS, dtype=np.float32)
        st = lib().eamg_gnn_params(self.h, _ptr(out))
        if st != EAMG_OK:
            raise EamgError(st, "eamg_gnn_params")
        return out

    def forward(self, X, edges, n):
        X, edges = self._graph(X, edges)
        z = np.zeros(X.shape[0], dtype=np.float32)
        st = lib().eamg_gnn_forward(self.h, X.shape[0], int(n), _ptr(X), _ptr(edges), _ptr(z))
        if st != EAMG_OK:
            raise EamgError(st, "eamg_gnn_forward")
        return z

    def loss_grad(self, X, edges, n, y, w):
        X, edges = self._graph(X, edges)
        y = np.ascontiguousarray(y, dtype=np.float32)
        w = np.ascontiguousarray(w, dtype=np.float32)
        loss = ctypes.c_double()
        g = np.zeros(GNN_PARAMS, dtype=np.float32)
        st = lib().eamg_gnn_loss_grad(self.h, X.shape[0], int(n), _ptr(X), _ptr(edges), _ptr(y),
                                      _ptr(w), ctypes.byref(loss), _ptr(g))
        if st != EAMG_OK:
            raise EamgError(st, "eamg_gnn_loss_grad")
        return loss.value, g

    def train(self, graphs, epochs, lr=3e-3):
        """graphs: list of (X, edges, n, y, w).  Returns the mean loss per epoch."""
        keep = []
        for X, edges, n, y, w in graphs:
            X, edges = self._graph(X, edges)
            keep.append((X, edges, int(n), np.ascontiguousarray(y, dtype=np.float32),
                         np.ascontiguousarray(w, dtype=np.float32)))
        k = len(keep)
        ms = np.array([g[0].shape[0] for g in keep], dtype=np.int64)
        ns = np.array([g[2] for g in keep], dtype=np.int32)
        arr = lambda i: (ctypes.c_void_p * k)(*[g[i].ctypes.data for g in keep])
        hist = np.zeros(epochs, dtype=np.float32)
        st = lib().eamg_gnn_train(self.h, k, _ptr(ms), _ptr(ns), arr(0), arr(1), arr(3), arr(4),
                                  int(epochs), float(lr), _ptr(hist))
        if st != EAMG_OK:
            raise EamgError(st, "eamg_gnn_train")
        return hist

    def close(self):
        if self.h is not None:
            lib().eamg_gnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eamg_coarsening_stats(h):
    ev, eg, sk = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    npass = ctypes.c_int32()
    st = lib().eamg_coarsening_stats(h, ctypes.byref(ev), ctypes.byref(eg), ctypes.byref(sk),
                                     ctypes.byref(npass))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_coarsening_stats")
    return dict(evaluated=ev.value, evaluated_g=eg.value, skipped=sk.value, sample_passes=npass.value)


def eamg_gnn_samples(h, k):
    """Recorded pass k: (X, edges, n, y, w)."""
    m, n = ctypes.c_int64(), ctypes.c_int32()
    st = lib().eamg_gnn_samples(h, int(k), ctypes.byref(m), ctypes.byref(n), None, None, None, None)
    if st != EAMG_OK:
        raise EamgError(st, "eamg_gnn_samples")
    X = np.zeros((m.value, GNN_FEATURES), dtype=np.float32)
    edges = np.zeros((m.value, 2), dtype=np.int32)
    y = np.zeros(m.value, dtype=np.float32)
    w = np.zeros(m.value, dtype=np.float32)
    st = lib().eamg_gnn_samples(h, int(k), ctypes.byref(m), ctypes.byref(n), _ptr(X), _ptr(edges),
                                _ptr(y), _ptr(w))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_gnn_samples")
    return X, edges, n.value, y, w


def eamg_autotune(h, panel_width=0, stream=None):
    """Tune launch shapes on the hierarchy; returns (ms before, ms after) of the tuned kernels."""
    b, a = ctypes.c_double(), ctypes.c_double()
    st = lib().eamg_autotune(h, int(panel_width), _stream(stream), ctypes.byref(b), ctypes.byref(a))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_autotune")
    return b.value, a.value


def eamg_vcycle(h, r, z, precision=EAMG_PRECOND_VCYCLE, stream=None):
    st = lib().eamg_vcycle(h, _dptr(r), _dptr(z), int(precision), _stream(stream))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_vcycle")


def eamg_vcycle_noalloc(h, r, z, precision=EAMG_PRECOND_VCYCLE, stream=None):
    """z = V(r) without allocation or synchronization (r, z: float64 device tensors)."""
    st = lib().eamg_vcycle_noalloc(h, _dptr(r), _dptr(z), int(precision), _stream(stream))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_vcycle_noalloc")


def eamg_stats(h):
    nl = ctypes.c_int32()
    ns = np.zeros(64, dtype=np.int64)
    nz = np.zeros(64, dtype=np.int64)
    vc, oc = ctypes.c_double(), ctypes.c_double()
    st = lib().eamg_stats(h, ctypes.byref(nl), _ptr(ns), _ptr(nz), ctypes.byref(vc), ctypes.byref(oc))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_stats")
    return dict(n_levels=nl.value, n=ns[:nl.value].tolist(), nnzb=nz[:nl.value].tolist(),
                vc=vc.value, oc=oc.value)


def eamg_level_info_get(h, level):
    info = eamg_level_info()
    st = lib().eamg_level_info_get(h, level, ctypes.byref(info))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_level_info_get")
    return {f: getattr(info, f) for f, _ in eamg_level_info._fields_}


def eamg_export_level(h, level):
    """Natural-order host copies of one level: agg, P (rowptr, col, val), A (...), color."""
    li = eamg_level_info_get(h, level)
    n, bs, kc = li["n"], li["bs"], li["k_coarse"]
    out = dict(info=li,
               agg=np.zeros(n, np.int32), color=np.zeros(n, np.int32),
               P_rowptr=np.zeros(n + 1, np.int32), P_col=np.zeros(max(li["nnzb_P"], 1), np.int32),
               P_val=np.zeros(max(li["nnzb_P"] * bs * kc, 1)),
               A_rowptr=np.zeros(n + 1, np.int32), A_col=np.zeros(li["nnzb_A"], np.int32),
               A_val=np.zeros(li["nnzb_A"] * bs * bs))
    st = lib().eamg_export_level(h, level, _ptr(out["agg"]), _ptr(out["P_rowptr"]),
                                 _ptr(out["P_col"]), _ptr(out["P_val"]), _ptr(out["A_rowptr"]),
                                 _ptr(out["A_col"]), _ptr(out["A_val"]), _ptr(out["color"]))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_export_level")
    out["P_col"] = out["P_col"][:li["nnzb_P"]]
    out["P_val"] = out["P_val"][:li["nnzb_P"] * bs * kc].reshape(-1, bs, kc) if kc else None
    out["A_val"] = out["A_val"].reshape(-1, bs, bs)
    return out


def eamg_traffic_model(h, precision=EAMG_PRECOND_VCYCLE):
    v, it = ctypes.c_double(), ctypes.c_double()
    st = lib().eamg_traffic_model(h, int(precision), ctypes.byref(v), ctypes.byref(it))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_traffic_model")
    return v.value, it.value


def eamg_solve_coefficients(h, max_entries=100000):
    """(alpha, beta) of the last single-vector solve on h, one entry per CG iteration."""
    a = np.zeros(max_entries)
    b = np.zeros(max_entries)
    n = ctypes.c_int32()
    st = lib().eamg_solve_coefficients(h, max_entries, _ptr(a), _ptr(b), ctypes.byref(n))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_solve_coefficients")
    m = min(n.value, max_entries)
    return a[:m].copy(), b[:m].copy()


def eamg_setup_phases(h, max_entries=64):
    """[(name, seconds, where)] with where "host", "device" or "copy"."""
    buf = (eamg_setup_phase * max_entries)()
    n = ctypes.c_int32()
    st = lib().eamg_setup_phases(h, max_entries, buf, ctypes.byref(n))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_setup_phases")
    names = {0: "host", 1: "device", 2: "copy"}
    return [(buf[i].name.decode(), buf[i].seconds, names[buf[i].where])
            for i in range(min(n.value, max_entries))]


def eamg_dense_tail(h):
    """(first level applied as the dense tail or -1, its dofs)."""
    lvl, dofs = ctypes.c_int32(), ctypes.c_int32()
    st = lib().eamg_dense_tail(h, ctypes.byref(lvl), ctypes.byref(dofs))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_dense_tail")
    return lvl.value, dofs.value


def eamg_profile_enable(h, on=True):
    st = lib().eamg_profile_enable(h, int(on))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_profile_enable")


def eamg_profile_read(h, max_entries=64):
    """Per-kernel records since enabling: list of dicts sorted by total time."""
    buf = (eamg_kernel_stat * max_entries)()
    n = ctypes.c_int32()
    st = lib().eamg_profile_read(h, max_entries, buf, ctypes.byref(n))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_profile_read")
    return [dict(name=buf[i].name.decode(), launches=buf[i].launches, total_ms=buf[i].total_ms,
                 bytes=buf[i].bytes) for i in range(min(n.value, max_entries))]


def eamg_destroy(h):
    if h is not None:
        lib().eamg_destroy(h)


def eamg_host_match(k, coords, edges, E, M, vd=None, params=None):
    """Host-only successive matching of one level; returns (agg, nc, coarse_coords, margin)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n = coords.shape[0]
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    E = np.ascontiguousarray(E, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    vdm = None if vd is None else np.ascontiguousarray(vd, dtype=np.uint8)
    agg = np.zeros(n, np.int32)
    cc = np.zeros((max(n, 1), 3))
    nc = ctypes.c_int32()
    margin = ctypes.c_double()
    st = lib().eamg_host_match(k, n, _ptr(coords), edges.shape[0], _ptr(edges), _ptr(E), _ptr(M),
                               _ptr(vdm), ctypes.byref(params) if params is not None else None,
                               _ptr(agg), ctypes.byref(nc), _ptr(cc), ctypes.byref(margin))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_host_match")
    return agg, nc.value, cc[:nc.value], margin.value


def eamg_criteria_eval(k, coords, edges, E, M, pairs, unions, tau=1e-10, use_device=True,
                       stream=None):
    """mu_b of each pair (m x 2) and mu_g of each union (u x 4, ascending, -1 padded) of one
    auxiliary level, by the GPU kernels (use_device) or the host code; returns (mub, mug)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n = coords.shape[0]
    edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    E = np.ascontiguousarray(E, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    unions = np.ascontiguousarray(unions, dtype=np.int32).reshape(-1, 4)
    mub = np.zeros(pairs.shape[0])
    mug = np.zeros(unions.shape[0])
    st = lib().eamg_criteria_eval(k, n, _ptr(coords), edges.shape[0], _ptr(edges), _ptr(E), _ptr(M),
                                  pairs.shape[0], _ptr(pairs), unions.shape[0], _ptr(unions),
                                  float(tau), int(bool(use_device)),
                                  _stream(stream) if use_device else None, _ptr(mub), _ptr(mug))
    if st != EAMG_OK:
        raise EamgError(st, "eamg_criteria_eval")
    return mub, mug


class Hierarchy:
    """Owning wrapper: setup on construction, solve(b) -> x on device tensors."""

    def __init__(self, dim, coords, row_ptr, col_idx, vals, dirichlet=None, params=None,
                 stream=None, **kw):
        self.dim = dim
        self.n_dofs = np.asarray(coords).shape[0] * dim
        self.h = None
        self.h = eamg_setup(dim, coords, row_ptr, col_idx, vals, dirichlet, params, stream, **kw)
        _OPEN.add(self)

    def solve(self, b, x=None, **kw):
        import torch
        if x is None:
            x = torch.zeros_like(b)
        st, info = eamg_solve(self.h, b, x, **kw)
        info["status"] = st
        return x, info

    def solve_batch(self, B, X=None, **kw):
        import torch
        if X is None:
            X = torch.zeros_like(B)
        st, infos = eamg_solve_batch(self.h, B, X, **kw)
        return X, st, infos

    def stats(self):
        return eamg_stats(self.h)

    def export(self, level):
        return eamg_export_level(self.h, level)

    def close(self):
        if self.h is not None:
            eamg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Fused:
    """Owning wrapper of a fused hierarchy (eamg_fuse) over Hierarchy objects; it keeps them
    referenced while it is open."""

    def __init__(self, hierarchies, dense_tail_dofs=0, stream=None):
        self.parts = list(hierarchies)
        self.dense_tail_dofs = int(dense_tail_dofs)
        self.h = None
        self.h = eamg_fuse([p.h for p in self.parts], dense_tail_dofs, stream)
        _OPEN.add(self)

    def solve(self, bs, xs=None, **kw):
        import torch
        if xs is None:
            xs = [torch.zeros_like(b) for b in bs]
        st, infos = eamg_solve_fused(self.h, bs, xs, **kw)
        return xs, st, infos

    def close(self):
        if self.h is not None:
            eamg_destroy(self.h)
            self.h = None
        self.parts = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
