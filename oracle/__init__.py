"""Python view of the CPU oracle (``liblgmg_oracle.so``).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH: only the test suite,
``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg import this.
The oracle is plain C (``lgmg_oracle.c``), fp64, and shares no code with the
GPU library.  The tests use its single-threaded build; the benchmark's CPU
baseline also times the OpenMP build, which computes identical bits.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblgmg_oracle.so")
# the same source built with -fopenmp: row-parallel loops, identical results;
# used for the benchmark's CPU timing baseline
OMP_LIB_PATH = os.path.join(_HERE, "liblgmg_oracle_omp.so")
SRC = os.path.join(_HERE, "lgmg_oracle.c")

AGG, ELIM, COARSEST = 0, 1, 2
STATUS = {0: "ok", 1: "bad argument", 2: "invalid graph", 3: "disconnected", 4: "out of memory",
          6: "not converged", 8: "exact-sum range exceeded"}


def build(verbose=False):
    """Compile the oracle with gcc (strict IEEE: no contraction, no fast-math),
    single-threaded and with OpenMP."""
    base = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-Wall", "-Wno-unused-function"]
    for extra, out in (([], LIB_PATH), (["-fopenmp"], OMP_LIB_PATH)):
        cmd = base + extra + [SRC, "-o", out, "-lm"]
        if not extra:
            cmd.insert(len(base), "-Wno-unknown-pragmas")
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
    return LIB_PATH


class Opts(C.Structure):
    _fields_ = [
        ("elim_enable", C.c_int32),
        ("elim_max_degree", C.c_int32),
        ("elim_min_fraction", C.c_double),
        ("agg_iters", C.c_int32),
        ("agg_filter_base", C.c_double),
        ("seed_votes", C.c_int32),
        ("tv_sweeps", C.c_int32),
        ("tv_omega", C.c_double),
        ("cheb_degree", C.c_int32),
        ("cheb_lo", C.c_double),
        ("cheb_hi", C.c_double),
        ("eig_iters", C.c_int32),
        ("coarsest_nnz", C.c_int64),
        ("max_levels", C.c_int32),
        ("cycle", C.c_int32),
        ("hash_mode", C.c_int32),
        ("seed", C.c_uint64),
        ("elim_passes", C.c_int32),
    ]


_libs = {}

_P = C.c_void_p
_I32, _I64, _U64, _D = C.c_int32, C.c_int64, C.c_uint64, C.c_double


def lib(threaded=False):
    """The single-threaded oracle, or (threaded=True) the OpenMP build."""
    if threaded in _libs:
        return _libs[threaded]
    path = OMP_LIB_PATH if threaded else LIB_PATH
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
        build()
    L = C.CDLL(path)
    sig = {
        "lgo_threads": (_I32, []),
        "lgo_default_opts": (None, [_P]),
        "lgo_mix64": (_U64, [_U64]),
        "lgo_hash": (_U64, [_I64, _I32]),
        "lgo_tv": (_D, [_U64, _I32, _I32, _I64]),
        "lgo_xs_term": (C.c_int, [_D, _P, _P]),
        "lgo_xs_round": (_D, [_I64, _U64]),
        "lgo_xsum": (C.c_int, [_P, _I64, _P]),
        "lgo_validate": (C.c_int, [_I64, _P, _P, _P]),
        "lgo_diag": (C.c_int, [_I64, _P, _P, _P, _P]),
        "lgo_elim_select": (_I64, [_I64, _P, _P, _I32, _I32, _P, _P]),
        "lgo_elim_build": (_I64, [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _I64]),
        "lgo_soc": (C.c_int, [_I64, _P, _P, _P, _P, _P, _I32, _P, _P]),
        "lgo_aggregate": (_I64, [_I64, _P, _P, _P, _P, _P, _P, _P, _P]),
        "lgo_galerkin": (_I64, [_I64, _P, _P, _P, _P, _I64, _P, _P, _P, _P, _I64]),
        "lgo_lanczos_lmax": (_D, [_I64, _P, _P, _P, _P, _I32, _U64, _I32]),
        "lgo_tridiag_max": (_D, [_P, _P, _I32]),
        "lgo_pinv_dense": (C.c_int, [_I64, _P, _P, _P, _P, _P]),
        "lgo_cheb_apply": (C.c_int, [_I64, _P, _P, _P, _P, _D, _P, _P, _P, _I32]),
        "lgo_setup": (C.c_int, [_I64, _P, _P, _P, _P, C.POINTER(_P)]),
        "lgo_free": (None, [_P]),
        "lgo_num_levels": (_I32, [_P]),
        "lgo_level_info": (C.c_int, [_P, _I32, _P, _P, _P, _P, _P]),
        "lgo_level_csr": (C.c_int, [_P, _I32, _P, _P, _P, _P]),
        "lgo_level_map": (C.c_int, [_P, _I32, _P]),
        "lgo_level_elim": (C.c_int, [_P, _I32, _P]),
        "lgo_level_soc": (C.c_int, [_P, _I32, _P, _P]),
        "lgo_level_votes": (C.c_int, [_P, _I32, _P, _P, _P]),
        "lgo_coarsest_pinv": (C.c_int, [_P, _P]),
        "lgo_cycle_work": (_D, [_P]),
        "lgo_cycle": (C.c_int, [_P, _P, _P]),
        "lgo_level_cycle": (C.c_int, [_P, _I32, _P, _P]),
        "lgo_level_fcg2": (C.c_int, [_P, _I32, _P, _P]),
        "lgo_spmv": (C.c_int, [_P, _I32, _P, _P]),
        "lgo_solve": (C.c_int, [_P, _P, _P, _D, _I32, _P, _P, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _libs[threaded] = L
    return L


def threads(threaded=False):
    """Threads the chosen build's row-parallel loops use."""
    return int(lib(threaded).lgo_threads())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def default_opts(**kw):
    o = Opts()
    lib().lgo_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _graph_arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.float64)
    return rp, col, w


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


# ---------------------------------------------------------------- primitives

def mix64(z):
    return int(lib().lgo_mix64(C.c_uint64(z & (2**64 - 1))))


def vertex_hash(i, mode=0):
    return int(lib().lgo_hash(i, mode))


def tv(seed, level, k, i):
    return float(lib().lgo_tv(seed, level, k, i))


def xs_term(v):
    hi, lo = C.c_int64(), C.c_uint64()
    st = lib().lgo_xs_term(float(v), C.byref(hi), C.byref(lo))
    return st, (hi.value << 64) | lo.value


def xs_round(s):
    s &= (1 << 128) - 1
    hi = s >> 64
    if hi >= 1 << 63:
        hi -= 1 << 64
    return float(lib().lgo_xs_round(hi, s & (2**64 - 1)))


def xsum(terms):
    t = np.ascontiguousarray(terms, dtype=np.float64)
    out = C.c_double()
    st = lib().lgo_xsum(_ptr(t), t.shape[0], C.byref(out))
    return st, out.value


def validate(g):
    rp, col, w = _graph_arrays(g)
    return int(lib().lgo_validate(g.n, _ptr(rp), _ptr(col), _ptr(w)))


def diag(g):
    rp, col, w = _graph_arrays(g)
    d = np.empty(g.n)
    st = lib().lgo_diag(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(d))
    if st:
        raise OracleError(st, "diag")
    return d


def elim_select(g, max_degree=4, hash_mode=0):
    rp, col, _ = _graph_arrays(g)
    z = np.empty(g.n, dtype=np.int32)
    F = np.empty(g.n, dtype=np.uint8)
    cnt = lib().lgo_elim_select(g.n, _ptr(rp), _ptr(col), max_degree, hash_mode, _ptr(z), _ptr(F))
    return int(cnt), z, F.astype(bool)


def elim_build(g, F, d=None):
    """Schur complement onto C = V \\ F.  Returns (cidx, coarse Graph-like tuple, cd)."""
    import graphgen

    rp, col, w = _graph_arrays(g)
    d = diag(g) if d is None else np.ascontiguousarray(d, dtype=np.float64)
    F8 = np.ascontiguousarray(F, dtype=np.uint8)
    nf = int(F8.sum())
    nc = g.n - nf
    deg = np.diff(rp)[F8.astype(bool)].astype(np.int64)
    cap = g.nnz + int(np.sum(deg * (deg - 1))) + 1  # an eliminated vertex of degree k adds <= k(k-1) entries
    cidx = np.empty(g.n, dtype=np.int32)
    crp = np.zeros(nc + 1, dtype=np.int64)
    ccol = np.empty(cap, dtype=np.int32)
    cw = np.empty(cap)
    cd = np.empty(nc)
    m = lib().lgo_elim_build(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(d), _ptr(F8), _ptr(cidx),
                             _ptr(crp), _ptr(ccol), _ptr(cw), _ptr(cd), cap)
    if m < 0:
        raise OracleError(-m, "elim_build")
    return cidx, graphgen.Graph(nc, crp, ccol[:m].copy(), cw[:m].copy()), cd


def soc(g, opts=None, level=0, d=None):
    rp, col, w = _graph_arrays(g)
    opts = opts or default_opts()
    d = diag(g) if d is None else np.ascontiguousarray(d, dtype=np.float64)
    X = np.empty((g.n, 4))
    S = np.empty(g.nnz)
    st = lib().lgo_soc(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(d), C.byref(opts), level, _ptr(X),
                       _ptr(S))
    if st:
        raise OracleError(st, "soc")
    return X, S


def aggregate(g, S, opts=None):
    """Voting aggregation on strengths S (one per stored edge of g)."""
    rp, col, _ = _graph_arrays(g)
    opts = opts or default_opts()
    S = np.ascontiguousarray(S, dtype=np.float64)
    state = np.empty(g.n, dtype=np.int32)
    idx = np.empty(g.n, dtype=np.int32)
    votes = np.empty(g.n, dtype=np.int32)
    agg = np.empty(g.n, dtype=np.int32)
    nc = lib().lgo_aggregate(g.n, _ptr(rp), _ptr(col), _ptr(S), C.byref(opts), _ptr(state),
                             _ptr(idx), _ptr(votes), _ptr(agg))
    return int(nc), agg, state, idx, votes


def galerkin(g, agg, nc):
    import graphgen

    rp, col, w = _graph_arrays(g)
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    cap = g.nnz + 1
    crp = np.zeros(nc + 1, dtype=np.int64)
    ccol = np.empty(cap, dtype=np.int32)
    cw = np.empty(cap)
    cd = np.empty(nc)
    m = lib().lgo_galerkin(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(agg), nc, _ptr(crp),
                           _ptr(ccol), _ptr(cw), _ptr(cd), cap)
    if m < 0:
        raise OracleError(-m, "galerkin")
    return graphgen.Graph(nc, crp, ccol[:m].copy(), cw[:m].copy()), cd


def lanczos_lmax(g, steps=10, seed=12345, level=0, d=None):
    rp, col, w = _graph_arrays(g)
    d = diag(g) if d is None else np.ascontiguousarray(d, dtype=np.float64)
    return float(lib().lgo_lanczos_lmax(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(d), steps, seed,
                                        level))


def tridiag_max(alpha, beta):
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    if b.shape[0] == 0:
        b = np.zeros(1)
    return float(lib().lgo_tridiag_max(_ptr(a), _ptr(b), a.shape[0]))


def pinv_dense(g, d=None):
    rp, col, w = _graph_arrays(g)
    d = diag(g) if d is None else np.ascontiguousarray(d, dtype=np.float64)
    out = np.empty((g.n, g.n))
    st = lib().lgo_pinv_dense(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(d), _ptr(out))
    if st:
        raise OracleError(st, "pinv_dense")
    return out


def cheb_apply(g, lmax, x, b, opts=None, x_is_zero=False, d=None):
    rp, col, w = _graph_arrays(g)
    opts = opts or default_opts()
    d = diag(g) if d is None else np.ascontiguousarray(d, dtype=np.float64)
    x = np.array(x, dtype=np.float64, copy=True)
    b = np.ascontiguousarray(b, dtype=np.float64)
    lib().lgo_cheb_apply(g.n, _ptr(rp), _ptr(col), _ptr(w), _ptr(d), lmax, C.byref(opts), _ptr(x),
                         _ptr(b), int(bool(x_is_zero)))
    return x


# ----------------------------------------------------------------- hierarchy

class Level:
    def __init__(self, type_, n, nnz, nc, lmax):
        self.type, self.n, self.nnz, self.nc, self.lmax = type_, n, nnz, nc, lmax


class Hierarchy:
    """Oracle hierarchy built by ``lgo_setup``; all exports are numpy copies."""

    def __init__(self, g, opts=None, threaded=False):
        self.opts = opts or default_opts()
        self._L = lib(threaded)
        rp, col, w = _graph_arrays(g)
        h = C.c_void_p()
        st = self._L.lgo_setup(g.n, _ptr(rp), _ptr(col), _ptr(w), C.byref(self.opts), C.byref(h))
        if st:
            raise OracleError(st, "setup")
        self._h = h
        self.n = g.n

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                self._L.lgo_free(h)
            except Exception:
                pass
            self._h = None

    @property
    def num_levels(self):
        return int(self._L.lgo_num_levels(self._h))

    def level(self, l):
        t, n, nnz, nc, lm = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64(), C.c_double()
        st = self._L.lgo_level_info(self._h, l, C.byref(t), C.byref(n), C.byref(nnz), C.byref(nc),
                                  C.byref(lm))
        if st:
            raise OracleError(st, "level_info")
        return Level(t.value, n.value, nnz.value, nc.value, lm.value)

    def levels(self):
        return [self.level(l) for l in range(self.num_levels)]

    def csr(self, l):
        import graphgen

        L = self.level(l)
        rp = np.empty(L.n + 1, dtype=np.int64)
        col = np.empty(max(L.nnz, 1), dtype=np.int32)
        w = np.empty(max(L.nnz, 1))
        d = np.empty(L.n)
        self._L.lgo_level_csr(self._h, l, _ptr(rp), _ptr(col), _ptr(w), _ptr(d))
        return graphgen.Graph(L.n, rp, col[:L.nnz].copy(), w[:L.nnz].copy()), d

    def map(self, l):
        L = self.level(l)
        out = np.empty(L.n, dtype=np.int32)
        st = self._L.lgo_level_map(self._h, l, _ptr(out))
        if st:
            raise OracleError(st, "level_map")
        return out

    def elim_z(self, l):
        L = self.level(l)
        out = np.empty(L.n, dtype=np.int32)
        st = self._L.lgo_level_elim(self._h, l, _ptr(out))
        if st:
            raise OracleError(st, "level_elim")
        return out

    def soc(self, l):
        L = self.level(l)
        X = np.empty((L.n, 4))
        S = np.empty(max(L.nnz, 1))
        st = self._L.lgo_level_soc(self._h, l, _ptr(X), _ptr(S))
        if st:
            raise OracleError(st, "level_soc")
        return X, S[:L.nnz].copy()

    def votes(self, l):
        L = self.level(l)
        s = np.empty(L.n, dtype=np.int32)
        i = np.empty(L.n, dtype=np.int32)
        v = np.empty(L.n, dtype=np.int32)
        st = self._L.lgo_level_votes(self._h, l, _ptr(s), _ptr(i), _ptr(v))
        if st:
            raise OracleError(st, "level_votes")
        return s, i, v

    def coarsest_pinv(self):
        n = self.level(self.num_levels - 1).n
        out = np.empty((n, n))
        self._L.lgo_coarsest_pinv(self._h, _ptr(out))
        return out

    def cycle_work(self):
        return float(self._L.lgo_cycle_work(self._h))

    def cycle(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(self.n)
        self._L.lgo_cycle(self._h, _ptr(b), _ptr(x))
        return x

    def level_cycle(self, l, b):
        """Algorithm 1 started on level l with zero initial guess (test hook)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty_like(b)
        st = self._L.lgo_level_cycle(self._h, l, _ptr(b), _ptr(x))
        if st:
            raise OracleError(st, "level_cycle")
        return x

    def level_fcg2(self, l, b):
        """The K-cycle's inner solve on level l: two flexible-CG steps
        preconditioned by the cycle from level l (test hook)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty_like(b)
        st = self._L.lgo_level_fcg2(self._h, l, _ptr(b), _ptr(x))
        if st:
            raise OracleError(st, "level_fcg2")
        return x

    def spmv(self, l, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        self._L.lgo_spmv(self._h, l, _ptr(x), _ptr(y))
        return y

    def solve(self, b, rtol=1e-8, max_iter=500):
        """Single right-hand side.  Returns (x, status, iters, rel_residual, work_units)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(self.n)
        it, rel, work = C.c_int32(), C.c_double(), C.c_double()
        st = self._L.lgo_solve(self._h, _ptr(b), _ptr(x), rtol, max_iter, C.byref(it), C.byref(rel),
                             C.byref(work))
        return x, int(st), it.value, rel.value, work.value


def eigs_dense(g, nev):
    """The nev smallest nonzero eigenvalues of L = D - A of a connected graph,
    ascending, with unit eigenvectors (columns): the definition itself, from
    the dense matrix (Section 2.1's eigensystem; its first vector is the
    Fiedler vector).  Small graphs only."""
    n = g.n
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    L = np.zeros((n, n))
    np.add.at(L, (rows, g.col), -g.w)
    L[np.arange(n), np.arange(n)] = np.bincount(rows, weights=g.w, minlength=n)
    lam, V = np.linalg.eigh(L)
    return lam[1:nev + 1], V[:, 1:nev + 1]
