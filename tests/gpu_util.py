"""Helpers shared by the GPU tests: run the HIP library and the CPU oracle on
the same seeded inputs and compare them."""

import sys

import numpy as np

import graphgen as gg
import oracle
import paper_1705_06266_amd.lgmg as lg


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch

    return torch.device("cuda:0")


def to_dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a)).to(torch_dev())


def gpu_setup(g, device_arrays=True, **opts):
    o = lg.lg_default_opts(**opts)
    if device_arrays:
        return lg.lg_setup(to_dev(g.row_ptr), to_dev(g.col), to_dev(g.w), o)
    return lg.lg_setup(g.row_ptr, g.col, g.w, o)


def oracle_opts(gpu_opts):
    names = [f for f, _ in oracle.Opts._fields_]
    return oracle.default_opts(**{k: getattr(gpu_opts, k) for k in names})


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def compare_hierarchies(hg, ho, setup_data=False):
    """Bit-for-bit comparison of every level: structure, values, decisions."""
    sg = lg.lg_hierarchy_stats(hg)
    so = ho.levels()
    assert [s["type"] for s in sg] == [L.type for L in so], "level types differ"
    assert [s["n"] for s in sg] == [L.n for L in so]
    assert [s["nnz"] for s in sg] == [L.nnz for L in so]
    for l, (a, b) in enumerate(zip(sg, so)):
        rp, col, w, d, mp = lg.lg_export_level(hg, l)
        go, do = ho.csr(l)
        assert np.array_equal(rp, go.row_ptr), f"level {l} row_ptr"
        assert np.array_equal(col, go.col), f"level {l} col"
        assert np.array_equal(bits(w), bits(go.w)), f"level {l} weights"
        assert np.array_equal(bits(d), bits(do)), f"level {l} diagonal"
        if a["type"] != oracle.COARSEST:
            assert a["nc"] == b.nc
            assert np.array_equal(mp, ho.map(l)), f"level {l} map"
        if a["type"] == oracle.AGG:
            # same exact-sum Lanczos steps; the two tridiagonal eigensolvers differ in ulps
            assert abs(a["lmax"] - b.lmax) <= 1e-12 * abs(b.lmax), f"level {l} lmax"
        if setup_data and a["type"] == oracle.AGG:
            sd = lg.lg_export_setup_data(hg, l)
            Xo, So = ho.soc(l)
            assert np.array_equal(bits(sd["X"]), bits(Xo)), f"level {l} test vectors"
            assert np.array_equal(bits(sd["S"]), bits(So)), f"level {l} strengths"
            st, ix, vo = ho.votes(l)
            assert np.array_equal(sd["state"], st), f"level {l} states"
            assert np.array_equal(sd["idx"], ix), f"level {l} roots"
            assert np.array_equal(sd["votes"], vo), f"level {l} votes"
        if setup_data and a["type"] == oracle.ELIM:
            sd = lg.lg_export_setup_data(hg, l, what=("z",))
            assert np.array_equal(sd["z"], ho.elim_z(l)), f"level {l} elimination product"
    Pg = lg.lg_export_coarsest(hg)
    Po = ho.coarsest_pinv()
    scale = max(np.abs(Po).max(), 1e-300)
    assert np.abs(Pg - Po).max() <= 1e-9 * scale, "coarsest pseudo-inverse"
    return sg


def dense_laplacian_norm(g, x):
    """sqrt(x^T L x) for a host graph."""
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    diff = x[rows] - x[g.col]
    return np.sqrt(0.5 * np.sum(g.w * diff * diff))


def laplacian_apply(g, x):
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    d = np.bincount(rows, weights=g.w, minlength=g.n)
    ax = np.bincount(rows, weights=g.w * x[g.col], minlength=g.n)
    return d * x - ax


def check_laplacian_level(rp, col, w, d):
    """Invariants of a graph Laplacian level: symmetric, positive off-diagonal
    weights (non-positive L entries), zero row sums to one rounding."""
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all(w > 0)
    assert np.all(col != rows)
    key = rows.astype(np.int64) * n + col
    tkey = col.astype(np.int64) * n + rows
    order = np.argsort(key)
    pos = np.searchsorted(key[order], tkey)
    assert np.all(pos < key.size)
    pos = order[pos]
    assert np.array_equal(key[pos], tkey), "not structurally symmetric"
    assert np.array_equal(bits(w[pos]), bits(w)), "weights not symmetric"
    s = np.bincount(rows, weights=w, minlength=n)
    assert np.all(np.abs(d - s) <= 1e-12 * np.maximum(d, 1e-300) + 0.0)
