"""Thin Python binding of liblgmg.so (see include/lgmg.h).

Argument marshalling only: every step of setup and solve runs in the HIP
library.  Device arrays are torch tensors on the current HIP device; streams
are torch streams.  Importing this module does not need a GPU; calling into
the library does.  If the library is not built the call fails loudly.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblgmg.so")

LG_OK, LG_E_ARG, LG_E_GRAPH, LG_E_DISCONNECTED, LG_E_NOMEM, LG_E_HIP = 0, 1, 2, 3, 4, 5
LG_E_NOT_CONVERGED, LG_E_BUSY, LG_E_RANGE = 6, 7, 8
LG_LEVEL_AGG, LG_LEVEL_ELIM, LG_LEVEL_COARSEST = 0, 1, 2
LG_CYCLE_V, LG_CYCLE_K = 1, 2
LG_FP64, LG_MIXED = 0, 1

EXPORTS = [
    "lg_default_opts", "lg_setup", "lg_solve", "lg_eigs", "lg_eigs_noalloc", "lg_cycle", "lg_spmv", "lg_hierarchy_stats",
    "lg_export_level", "lg_export_setup_data", "lg_export_coarsest", "lg_hierarchy_bytes",
    "lg_setup_ms", "lg_free", "lg_profile_enable", "lg_profile_read", "lg_profile_names",
    "lg_status_str", "lg_last_error",
    "lg_server_default_opts", "lg_server_create", "lg_server_add_graph", "lg_server_submit",
    "lg_server_wait", "lg_server_stats_get", "lg_server_free",
]


class lg_graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("w", C.c_void_p), ("on_device", C.c_int32)]


class lg_setup_opts(C.Structure):
    _fields_ = [
        ("elim_enable", C.c_int32), ("elim_max_degree", C.c_int32),
        ("elim_min_fraction", C.c_double), ("agg_iters", C.c_int32),
        ("agg_filter_base", C.c_double), ("seed_votes", C.c_int32), ("tv_sweeps", C.c_int32),
        ("tv_omega", C.c_double), ("cheb_degree", C.c_int32), ("cheb_lo", C.c_double),
        ("cheb_hi", C.c_double), ("eig_iters", C.c_int32), ("coarsest_nnz", C.c_int64),
        ("max_levels", C.c_int32), ("cycle", C.c_int32), ("hash_mode", C.c_int32),
        ("seed", C.c_uint64), ("precision", C.c_int32), ("max_rhs", C.c_int32),
        ("keep_setup_data", C.c_int32), ("validate", C.c_int32), ("graphs", C.c_int32),
        ("autotune", C.c_int32), ("elim_passes", C.c_int32), ("merge_path", C.c_int32),
        ("row_shift", C.c_int32), ("reorder", C.c_int32), ("col_unroll", C.c_int32),
    ]


class lg_level_stats(C.Structure):
    _fields_ = [("type", C.c_int32), ("n", C.c_int64), ("nnz", C.c_int64), ("nc", C.c_int64),
                ("lmax", C.c_double), ("n_hub", C.c_int64), ("lane_shift", C.c_int32),
                ("col_shift", C.c_int32), ("merge", C.c_int32), ("reordered", C.c_int32),
                ("col_unroll", C.c_int32)]


class lg_rhs_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_residual", C.c_double), ("work_units", C.c_double),
                ("wda", C.c_double)]


class lg_server_opts(C.Structure):
    _fields_ = [("workers", C.c_int32), ("max_batch_rhs", C.c_int32), ("hbm_budget", C.c_size_t),
                ("setup", lg_setup_opts)]


class lg_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("batched_columns", C.c_int64), ("setups", C.c_int64), ("evictions", C.c_int64),
                ("resident_bytes", C.c_size_t), ("budget_bytes", C.c_size_t),
                ("resident_graphs", C.c_int32), ("refills", C.c_int64)]


class LgError(RuntimeError):
    def __init__(self, code, where, detail=""):
        super().__init__(f"{where}: {status_str(code)} ({code}) {detail}".strip())
        self.code = code


_lib = None
_P, _I32, _I64, _D = C.c_void_p, C.c_int32, C.c_int64, C.c_double


def load():
    """The loaded library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    sig = {
        "lg_default_opts": (_I32, [_P]),
        "lg_setup": (_I32, [_P, _P, _P, C.POINTER(_P)]),
        "lg_solve": (_I32, [_P, _P, _P, _I32, _D, _I32, _P, _P]),
        "lg_cycle": (_I32, [_P, _P, _P, _I32, _P]),
        "lg_eigs": (_I32, [_P, _I32, _D, _I32, _P, _P, _P, _P, _P]),
        "lg_eigs_noalloc": (_I32, [_P, _I32, _D, _I32, _P, _P, _P, _P, _P]),
        "lg_spmv": (_I32, [_P, _I32, _P, _P, _I32, _P]),
        "lg_hierarchy_stats": (_I32, [_P, _P, _I32, _P]),
        "lg_export_level": (_I32, [_P, _I32, _P, _P, _P, _P, _P]),
        "lg_export_setup_data": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _P]),
        "lg_export_coarsest": (_I32, [_P, _P]),
        "lg_hierarchy_bytes": (C.c_size_t, [_P]),
        "lg_setup_ms": (_D, [_P]),
        "lg_free": (None, [_P]),
        "lg_profile_enable": (_I32, [C.c_char_p]),
        "lg_profile_read": (_I32, [_P, _P, _P]),
        "lg_profile_names": (C.c_char_p, []),
        "lg_status_str": (C.c_char_p, [_I32]),
        "lg_last_error": (C.c_char_p, []),
        "lg_server_default_opts": (_I32, [_P]),
        "lg_server_create": (_I32, [_P, C.POINTER(_P)]),
        "lg_server_add_graph": (_I32, [_P, _P, _P]),
        "lg_server_submit": (_I32, [_P, _I32, _P, _P, _I32, _D, _I32, _P]),
        "lg_server_wait": (_I32, [_P, _I64, _P, _P]),
        "lg_server_stats_get": (_I32, [_P, _P]),
        "lg_server_free": (None, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_str(code):
    try:
        return load().lg_status_str(code).decode()
    except Exception:
        return str(code)


def lg_last_error():
    return load().lg_last_error().decode()


def _check(code, where, ok=(LG_OK,)):
    if code not in ok:
        raise LgError(code, where, lg_last_error())
    return code


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())


def _stream(stream):
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def lg_default_opts(**overrides):
    o = lg_setup_opts()
    _check(load().lg_default_opts(C.byref(o)), "lg_default_opts")
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Hierarchy:
    """Owner of an lg_hierarchy*; freed with lg_free when collected."""

    def __init__(self, handle, n, opts):
        self._h = handle
        self.n = n
        self.opts = opts

    @property
    def handle(self):
        return self._h

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.lg_free(self._h)
            self._h = None


def lg_setup(row_ptr, col, w, opts=None, stream=None):
    """Build the hierarchy.  Arrays are host numpy or device torch tensors
    (int64 row_ptr, int32 col, float64 w), all on the same side."""
    on_device = not isinstance(row_ptr, np.ndarray)
    if not on_device:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        w = np.ascontiguousarray(w, dtype=np.float64)
        n = row_ptr.shape[0] - 1
        nnz = col.shape[0]
    else:
        n = row_ptr.numel() - 1
        nnz = col.numel()
    g = lg_graph(n, nnz, _ptr(row_ptr), _ptr(col), _ptr(w), 1 if on_device else 0)
    o = opts if opts is not None else lg_default_opts()
    h = C.c_void_p()
    _check(load().lg_setup(C.byref(g), C.byref(o), _stream(stream), C.byref(h)), "lg_setup")
    return Hierarchy(h, n, o)


def lg_solve(h, B, X=None, rtol=1e-8, max_iter=500, stream=None, allow_unconverged=False):
    """Solve L X = B - mean(B) for device float64 B of shape (n, k).
    Returns (X, infos, status)."""
    import torch

    if B.dim() == 1:
        B = B.unsqueeze(1)
    B = B.contiguous()
    k = B.shape[1]
    if X is None:
        X = torch.empty_like(B)
    info = (lg_rhs_info * k)()
    ok = (LG_OK, LG_E_NOT_CONVERGED) if allow_unconverged else (LG_OK,)
    st = _check(load().lg_solve(h.handle, _ptr(B), _ptr(X), k, rtol, max_iter, _stream(stream),
                                info), "lg_solve", ok)
    infos = [dict(iters=i.iters, rel_residual=i.rel_residual, work_units=i.work_units, wda=i.wda)
             for i in info]
    return X, infos, st


def lg_eigs(h, nev=1, tol=1e-8, max_iter=200, stream=None, allow_unconverged=False):
    """The nev smallest nonzero eigenpairs of L: (lambda, X, iters, resid, status)
    with lambda a numpy array and X a device float64 tensor of shape (n, nev)."""
    import torch

    X = torch.empty((h.n, nev), dtype=torch.float64, device=torch.device("cuda", torch.cuda.current_device()))
    lam = np.zeros(nev)
    res = np.zeros(nev)
    it = C.c_int32()
    ok = (LG_OK, LG_E_NOT_CONVERGED) if allow_unconverged else (LG_OK,)
    st = _check(load().lg_eigs(h.handle, nev, tol, max_iter, _ptr(X), _ptr(lam), C.byref(it),
                               _ptr(res), _stream(stream)), "lg_eigs", ok)
    return lam, X, it.value, res, st


def lg_eigs_noalloc(h, nev, X, tol=1e-8, max_iter=200, stream=None, allow_unconverged=False):
    """lg_eigs without device allocation inside the call: X (device float64,
    shape (n, nev)) is the caller's output; returns (lambda, iters, resid, status)."""
    lam = np.zeros(nev)
    res = np.zeros(nev)
    it = C.c_int32()
    ok = (LG_OK, LG_E_NOT_CONVERGED) if allow_unconverged else (LG_OK,)
    st = _check(load().lg_eigs_noalloc(h.handle, nev, tol, max_iter, _ptr(X), _ptr(lam),
                                       C.byref(it), _ptr(res), _stream(stream)),
                "lg_eigs_noalloc", ok)
    return lam, it.value, res, st


def lg_cycle(h, B, X=None, stream=None):
    """X = M B for one preconditioner cycle (device float64, shape (n, k))."""
    import torch

    if B.dim() == 1:
        B = B.unsqueeze(1)
    B = B.contiguous()
    if X is None:
        X = torch.empty_like(B)
    _check(load().lg_cycle(h.handle, _ptr(B), _ptr(X), B.shape[1], _stream(stream)), "lg_cycle")
    return X


def lg_spmv(h, level, X, Y, stream=None):
    """Y = L_level X (device float64, (n_l, k), k a power of two <= 32); asynchronous."""
    k = X.shape[1] if X.dim() == 2 else 1
    _check(load().lg_spmv(h.handle, level, _ptr(X), _ptr(Y), k, _stream(stream)), "lg_spmv")
    return Y


def lg_hierarchy_stats(h):
    nl = C.c_int32()
    _check(load().lg_hierarchy_stats(h.handle, None, 0, C.byref(nl)), "lg_hierarchy_stats")
    arr = (lg_level_stats * nl.value)()
    _check(load().lg_hierarchy_stats(h.handle, arr, nl.value, C.byref(nl)), "lg_hierarchy_stats")
    return [dict(type=s.type, n=s.n, nnz=s.nnz, nc=s.nc, lmax=s.lmax, n_hub=s.n_hub,
                 lane_shift=s.lane_shift, col_shift=s.col_shift, merge=s.merge,
                 reordered=s.reordered, col_unroll=s.col_unroll) for s in arr]


def lg_export_level(h, level):
    """Host copies of level `level`: (row_ptr, col, w, d, map or None)."""
    st = lg_hierarchy_stats(h)[level]
    rp = np.empty(st["n"] + 1, dtype=np.int64)
    col = np.empty(max(st["nnz"], 1), dtype=np.int32)
    w = np.empty(max(st["nnz"], 1))
    d = np.empty(st["n"])
    mp = None
    if st["type"] != LG_LEVEL_COARSEST:
        mp = np.empty(st["n"], dtype=np.int32)
    _check(load().lg_export_level(h.handle, level, _ptr(rp), _ptr(col), _ptr(w), _ptr(d),
                                  _ptr(mp)), "lg_export_level")
    return rp, col[:st["nnz"]].copy(), w[:st["nnz"]].copy(), d, mp


def lg_export_setup_data(h, level, what=("X", "S", "state", "idx", "votes")):
    st = lg_hierarchy_stats(h)[level]
    n, nnz = st["n"], st["nnz"]
    bufs = {
        "X": np.empty((n, 4)) if "X" in what else None,
        "S": np.empty(max(nnz, 1)) if "S" in what else None,
        "state": np.empty(n, dtype=np.int32) if "state" in what else None,
        "idx": np.empty(n, dtype=np.int32) if "idx" in what else None,
        "votes": np.empty(n, dtype=np.int32) if "votes" in what else None,
        "z": np.empty(n, dtype=np.int32) if "z" in what else None,
    }
    _check(load().lg_export_setup_data(h.handle, level, *[_ptr(bufs[k]) for k in
                                                          ("X", "S", "state", "idx", "votes",
                                                           "z")]), "lg_export_setup_data")
    if bufs["S"] is not None:
        bufs["S"] = bufs["S"][:nnz].copy()
    return {k: v for k, v in bufs.items() if v is not None}


def lg_export_coarsest(h):
    n = lg_hierarchy_stats(h)[-1]["n"]
    out = np.empty((n, n))
    _check(load().lg_export_coarsest(h.handle, _ptr(out)), "lg_export_coarsest")
    return out


def lg_hierarchy_bytes(h):
    return int(load().lg_hierarchy_bytes(h.handle))


def lg_setup_ms(h):
    return float(load().lg_setup_ms(h.handle))


def lg_profile_enable(family):
    _check(load().lg_profile_enable(family.encode() if family else None), "lg_profile_enable")


def lg_profile_read():
    n, ms, b = C.c_int64(), C.c_double(), C.c_double()
    _check(load().lg_profile_read(C.byref(n), C.byref(ms), C.byref(b)), "lg_profile_read")
    return n.value, ms.value, b.value


def lg_profile_names():
    return load().lg_profile_names().decode().split(",")


# --------------------------------------------------------------- solve server
class Server:
    """Continuous-batching solve server (lg_server_*).  Keeps the caller's
    tensors of every request alive until the request has been waited for."""

    def __init__(self, workers=4, max_batch_rhs=32, hbm_budget=0, **setup_overrides):
        o = lg_server_opts()
        _check(load().lg_server_default_opts(C.byref(o)), "lg_server_default_opts")
        o.workers, o.max_batch_rhs, o.hbm_budget = workers, max_batch_rhs, hbm_budget
        for k, v in setup_overrides.items():
            setattr(o.setup, k, v)
        self.opts = o
        h = C.c_void_p()
        _check(load().lg_server_create(C.byref(o), C.byref(h)), "lg_server_create")
        self.handle = h
        self._live = {}
        self._n = {}

    def add_graph(self, row_ptr, col, w):
        """Register a graph (host numpy or device torch arrays); returns its id."""
        on_device = not isinstance(row_ptr, np.ndarray)
        if not on_device:
            row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
            col = np.ascontiguousarray(col, dtype=np.int32)
            w = np.ascontiguousarray(w, dtype=np.float64)
            n, nnz = row_ptr.shape[0] - 1, col.shape[0]
        else:
            n, nnz = row_ptr.numel() - 1, col.numel()
        g = lg_graph(n, nnz, _ptr(row_ptr), _ptr(col), _ptr(w), 1 if on_device else 0)
        gid = C.c_int32()
        _check(load().lg_server_add_graph(self.handle, C.byref(g), C.byref(gid)), "lg_server_add_graph")
        self._n[gid.value] = n
        return gid.value

    def submit(self, graph_id, B, X=None, rtol=1e-8, max_iter=500):
        """Queue a solve for device float64 B of shape (n, k); returns a request id.
        B's values must be final (synchronise its stream first)."""
        import torch

        if B.dim() == 1:
            B = B.unsqueeze(1)
        B = B.contiguous()
        if X is None:
            X = torch.empty_like(B)
        rid = C.c_int64()
        _check(load().lg_server_submit(self.handle, graph_id, _ptr(B), _ptr(X), B.shape[1], rtol,
                                       max_iter, C.byref(rid)), "lg_server_submit")
        self._live[rid.value] = (B, X)
        return rid.value

    def wait(self, request_id, allow_unconverged=False):
        """Block until the request is done: (X, infos, status, latency_ms)."""
        B, X = self._live[request_id]
        info = (lg_rhs_info * B.shape[1])()
        lat = C.c_double()
        ok = (LG_OK, LG_E_NOT_CONVERGED) if allow_unconverged else (LG_OK,)
        try:
            st = _check(load().lg_server_wait(self.handle, request_id, info, C.byref(lat)),
                        "lg_server_wait", ok)
        finally:
            del self._live[request_id]
        infos = [dict(iters=i.iters, rel_residual=i.rel_residual, work_units=i.work_units,
                      wda=i.wda) for i in info]
        return X, infos, st, lat.value

    def stats(self):
        st = lg_server_stats()
        _check(load().lg_server_stats_get(self.handle, C.byref(st)), "lg_server_stats_get")
        return {f: getattr(st, f) for f, _ in lg_server_stats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            load().lg_server_free(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
