"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks one part of the oracle against something the paper or the
mathematics fixes: published generator outputs, exact rational arithmetic,
closed forms, dense linear algebra (numpy/scipy), brute-force characterisations
and hand-traced cases of Algorithms 2 and 3.  No GPU is used.
"""

import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_A(g):
    A = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    A[rows, g.col] = g.w
    return A


def dense_L(g, d=None):
    A = dense_A(g)
    return np.diag(A.sum(1) if d is None else d) - A


def sparse_A(g):
    return sp.csr_matrix((g.w, g.col, g.row_ptr), shape=(g.n, g.n))


SMALL_GRAPHS = [
    lambda: gg.grid2d(9, 7),
    lambda: gg.grid3d(4, 5, 3, weights="loguniform", seed=11),
    lambda: gg.gnp(120, 0.05, seed=3),
    lambda: gg.rmat(8, 8, seed=5),
    lambda: gg.chung_lu(600, seed=9, max_deg=80),
    lambda: gg.star(12),
    lambda: gg.path(17),
    lambda: gg.cycle(10),
]


# ------------------------------------------------------------ generators

def test_splitmix64_published_outputs():
    lines = open(os.path.join(GOLDEN, "splitmix64_seed0.txt")).read().splitlines()
    vals = [int(t, 16) for t in lines if t.startswith("0x")]
    assert len(vals) == 5
    assert [oracle.vertex_hash(i) for i in range(5)] == vals


def test_hash_identity_mode_and_bijection_sample():
    assert oracle.vertex_hash(7, 1) == 7
    hs = {oracle.vertex_hash(i) for i in range(5000)}
    assert len(hs) == 5000


def test_test_vectors_uniform_on_53bit_grid():
    xs = np.array([oracle.tv(3, 1, k, i) for k in range(4) for i in range(4000)])
    assert np.all(xs >= -1.0) and np.all(xs < 1.0)
    scaled = (xs + 1.0) * 2.0**52
    assert np.all(scaled == np.floor(scaled))
    assert abs(xs.mean()) < 0.02
    assert abs(xs.var() - 1.0 / 3.0) < 0.01
    # streams differ by level, vector index and seed
    assert oracle.tv(3, 1, 0, 5) != oracle.tv(3, 2, 0, 5)
    assert oracle.tv(3, 1, 0, 5) != oracle.tv(3, 1, 1, 5)
    assert oracle.tv(3, 1, 0, 5) != oracle.tv(4, 1, 0, 5)


# ------------------------------------------------------------ exact sums

def _exact_term(v):
    return round(Fraction(v) * 2**64)  # Fraction.__round__: nearest, ties to even


def _edge_values(rng):
    vals = list(rng.standard_normal(200) * 10.0 ** rng.integers(-22, 12, 200))
    # exact ties at the 2^-64 grid: odd multiples of 2^-65
    vals += [math.ldexp(2 * k + 1, -65) for k in range(-6, 6)]
    vals += [math.ldexp(3, -66), -math.ldexp(3, -66), math.ldexp(1, -66), 5e-324, -5e-324, 0.0]
    vals += [math.ldexp(1, 61), -math.ldexp(1, 61) + 1.0, 1e-20, 1.5e-19, 2.5e-19]
    return vals


def test_xs_term_is_nearest_integer_ties_to_even():
    rng = np.random.default_rng(0)
    for v in _edge_values(rng):
        st, t = oracle.xs_term(float(v))
        assert st == 0
        if t >= 1 << 127:
            t -= 1 << 128
        assert t == _exact_term(float(v)), v


def test_xs_term_range_guard():
    assert oracle.xs_term(2.0**63)[0] == 8
    assert oracle.xs_term(float("nan"))[0] == 8


def test_xs_round_is_correctly_rounded():
    rng = np.random.default_rng(1)
    cases = [0, 1, -1, (1 << 53) + 1, (1 << 54) + 2, (1 << 54) + 6, -(1 << 100) - 3]
    for _ in range(400):
        bits = int(rng.integers(1, 126))
        s = int(rng.integers(0, 2**62)) << max(0, bits - 62) | int(rng.integers(0, 2**20))
        s &= (1 << 126) - 1
        cases.append(s if rng.random() < 0.5 else -s)
    # halfway cases: 53 significant bits then exactly one half ulp
    for m in [(1 << 52) + 1, (1 << 52) + 2, (1 << 53) - 1]:
        cases.append((2 * m + 1) << 10)
    for s in cases:
        assert oracle.xs_round(s) == float(Fraction(s, 2**64)), s


def test_xsum_equals_fsum_for_grid_aligned_terms():
    rng = np.random.default_rng(2)
    for _ in range(50):
        n = int(rng.integers(1, 300))
        t = rng.standard_normal(n) * 10.0 ** rng.integers(-3, 9, n)
        t = np.where(np.abs(t) < 2.0**-10, 2.0**-10, t)  # exponent >= -11: on the 2^-64 grid
        st, s = oracle.xsum(t)
        assert st == 0
        assert s == math.fsum(t)


def test_xsum_is_order_independent():
    rng = np.random.default_rng(3)
    t = rng.standard_normal(1000) * 10.0 ** rng.integers(-25, 10, 1000)
    ref = oracle.xsum(t)[1]
    for _ in range(5):
        assert oracle.xsum(rng.permutation(t))[1] == ref
    exact = sum(_exact_term(float(v)) for v in t)
    assert ref == float(Fraction(exact, 2**64))


# ------------------------------------------------------------ validation

def test_validate_accepts_generated_graphs():
    for mk in SMALL_GRAPHS:
        assert oracle.validate(mk()) == 0


def test_validate_rejects_bad_graphs():
    g = gg.grid2d(4, 4)
    bad = g.copy()
    bad.w[3] *= 2.0  # asymmetric weight
    assert oracle.validate(bad) == 2
    bad = g.copy()
    bad.w[0] = -1.0
    assert oracle.validate(bad) == 2
    bad = g.copy()
    bad.w[0] = 0.0
    assert oracle.validate(bad) == 2
    bad = g.copy()
    bad.col[0] = 0  # self loop in row 0
    assert oracle.validate(bad) == 2
    bad = g.copy()
    bad.col[[1, 2]] = bad.col[[2, 1]]  # unsorted row
    assert oracle.validate(bad) == 2
    two = gg.from_edges(4, [0, 2], [1, 3])
    assert oracle.validate(two) == 3
    assert oracle.validate(gg.from_edges(1, [], [])) == 0


# ------------------------------------------------------------ diagonal

def test_diag_is_correctly_rounded_row_sum():
    g = gg.grid3d(6, 5, 4, weights="loguniform", seed=4)  # weights >= 1e-3: on the 2^-64 grid
    d = oracle.diag(g)
    for i in range(g.n):
        assert d[i] == math.fsum(g.w[g.row_ptr[i]:g.row_ptr[i + 1]])


# ------------------------------------------------------ elimination select

def test_elim_select_local_min_characterisation():
    for mk in SMALL_GRAPHS:
        g = mk()
        deg = g.degrees()
        cnt, z, F = oracle.elim_select(g)
        h = np.array([oracle.vertex_hash(i) for i in range(g.n)], dtype=object)
        for i in range(g.n):
            nb = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
            cands = [j for j in list(nb) + [i] if deg[j] <= 4]
            expect_z = min(cands, key=lambda j: h[j]) if cands else -1
            assert z[i] == expect_z
            local_min = deg[i] <= 4 and all(h[i] < h[j] for j in nb if deg[j] <= 4)
            assert F[i] == local_min
        assert cnt == F.sum()
        # F is an independent set
        rows = np.repeat(np.arange(g.n), deg)
        assert not np.any(F[rows] & F[g.col])


def test_elim_chain_sequential_hashes_eliminate_one_vertex():
    g = gg.path(40)
    cnt, z, F = oracle.elim_select(g, hash_mode=1)
    assert cnt == 1 and F[0]


def test_elim_chain_alternating_hashes_eliminate_every_other_vertex():
    n = 40
    # chain position p carries id p//2 (low) when p is even, n//2 + p//2 (high) when odd
    ids = np.array([p // 2 if p % 2 == 0 else n // 2 + p // 2 for p in range(n)])
    g = gg.from_edges(n, ids[:-1], ids[1:])
    cnt, z, F = oracle.elim_select(g, hash_mode=1)
    assert cnt == n // 2
    assert set(np.nonzero(F)[0]) == set(range(n // 2))


def test_elim_high_degree_vertices_are_not_candidates():
    g = gg.star(6)
    cnt, z, F = oracle.elim_select(g)
    assert not F[0] and F[1:].all() and cnt == 6
    assert z[0] == min(range(1, 7), key=oracle.vertex_hash)


# --------------------------------------------------- Schur complement level

def test_schur_leaf_elimination_deletes_the_edge():
    g = gg.from_edges(3, [0, 1], [1, 2], [2.0, 3.0])
    F = np.array([True, False, False])
    cidx, gc, cd = oracle.elim_build(g, F)
    assert list(cidx) == [-1, 0, 1]
    assert gc.nnz == 2 and np.all(gc.w == 3.0) and np.all(cd == 3.0)


def test_schur_degree_two_vertex_gives_series_edge():
    g = gg.path(3)
    cidx, gc, cd = oracle.elim_build(g, np.array([False, True, False]))
    assert list(gc.w) == [0.5, 0.5] and list(cd) == [0.5, 0.5]
    g = gg.from_edges(3, [0, 1], [1, 2], [2.0, 6.0])
    _, gc, _ = oracle.elim_build(g, np.array([False, True, False]))
    assert np.allclose(gc.w, 2.0 * 6.0 / 8.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("max_degree", [4, 6, 10])
def test_schur_matches_dense_block_formula_and_two_level_identity(max_degree):
    top = 0  # highest degree eliminated over the graphs
    for mk in SMALL_GRAPHS:
        g = mk()
        cnt, z, F = oracle.elim_select(g, max_degree=max_degree)
        if cnt == 0:
            continue
        assert np.all(g.degrees()[F] <= max_degree)
        top = max(top, int(g.degrees()[F].max()))
        cidx, gc, cd = oracle.elim_build(g, F)
        L = dense_L(g)
        Fi = np.nonzero(F)[0]
        Ci = np.nonzero(~F)[0]
        assert np.array_equal(cidx[Ci], np.arange(Ci.size))
        LFF = L[np.ix_(Fi, Fi)]
        assert np.allclose(LFF, np.diag(np.diag(LFF)))  # diagonal: F independent
        LFC = L[np.ix_(Fi, Ci)]
        schur = L[np.ix_(Ci, Ci)] - LFC.T @ np.diag(1.0 / np.diag(LFF)) @ LFC
        Lc = dense_L(gc, cd)
        scale = np.abs(schur).max()
        assert np.abs(Lc - schur).max() <= 1e-13 * scale
        # additive two-level form: x = P Lc^+ P^T b + [L_FF^-1 b_F; 0] solves L x = b
        P = np.zeros((g.n, Ci.size))
        P[Ci, np.arange(Ci.size)] = 1.0
        P[np.ix_(Fi, np.arange(Ci.size))] = -np.diag(1.0 / np.diag(LFF)) @ LFC
        rng = np.random.default_rng(0)
        b = rng.standard_normal(g.n)
        b -= b.mean()
        x = P @ np.linalg.pinv(schur) @ P.T @ b
        x[Fi] += b[Fi] / np.diag(LFF)
        assert np.linalg.norm(L @ x - b) <= 1e-9 * np.linalg.norm(b)
    assert top > 4 or max_degree == 4, "the degree bound above 4 eliminated nothing above 4"


# ------------------------------------------------------------------- SoC

def test_soc_test_vectors_follow_weighted_jacobi():
    g = gg.chung_lu(400, seed=2, max_deg=50)
    opts = oracle.default_opts()
    X, S = oracle.soc(g, opts, level=3)
    X0 = np.array([[oracle.tv(opts.seed, 3, k, i) for k in range(4)] for i in range(g.n)])
    A = sparse_A(g)
    d = np.asarray(A.sum(1)).ravel()
    w = opts.tv_omega
    Y = X0
    for _ in range(opts.tv_sweeps):
        Y = (1 - w) * Y + w * (A @ Y) / d[:, None]
    assert np.abs(X - Y).max() <= 1e-14


def test_soc_strength_invariants():
    for mk in SMALL_GRAPHS:
        g = mk()
        X, S = oracle.soc(g)
        assert np.all(S >= 0.0) and np.all(S <= 1.0 + 1e-15)
        # symmetric, bit for bit
        rows = np.repeat(np.arange(g.n), g.degrees())
        key = rows * g.n + g.col
        tkey = g.col.astype(np.int64) * g.n + rows
        order = np.argsort(key)
        pos = order[np.searchsorted(key[order], tkey)]
        assert np.array_equal(S, S[pos])
        assert S.max() == 1.0
        # Cauchy-Schwarz bound on the affinity of each edge
        nx = np.linalg.norm(X, axis=1)
        cos2 = (np.einsum("ij,ij->i", X[rows], X[g.col]) / (nx[rows] * nx[g.col])) ** 2
        assert np.all(S >= cos2 * (1 - 1e-12))  # S >= C because every row maximum is <= 1
        M = np.zeros(g.n)
        np.maximum.at(M, rows, cos2)
        expect = cos2 / np.maximum(M[rows], M[g.col])
        assert np.allclose(S, expect, rtol=1e-12, atol=1e-14)


def test_soc_single_edge_has_strength_one():
    g = gg.path(2)
    _, S = oracle.soc(g)
    assert list(S) == [1.0, 1.0]


# ----------------------------------------------------------- aggregation

def _uniform_S(g, value=1.0):
    return np.full(g.nnz, value)


def test_star_seed_threshold_is_at_least_eight():
    o1 = oracle.default_opts(agg_iters=1)
    for m, seed_after_one in [(7, False), (8, True), (9, True)]:
        g = gg.star(m)
        nc, agg, state, idx, votes = oracle.aggregate(g, _uniform_S(g), o1)
        assert votes[0] == m
        assert (state[0] == 2) == seed_after_one
    o2 = oracle.default_opts(agg_iters=2)
    assert oracle.aggregate(gg.star(8), _uniform_S(gg.star(8)), o2)[0] == 1
    assert oracle.aggregate(gg.star(7), _uniform_S(gg.star(7)), o2)[0] == 8


def test_filter_keeps_strength_equal_to_threshold():
    g = gg.star(8)
    o1 = oracle.default_opts(agg_iters=1)
    _, _, state, _, votes = oracle.aggregate(g, _uniform_S(g, 0.5), o1)
    assert votes[0] == 8 and state[0] == 2
    _, _, state, _, votes = oracle.aggregate(g, _uniform_S(g, 0.4999), o1)
    assert votes[0] == 0 and state[0] == 1


def test_path_hand_trace():
    # Hand trace (all strengths 1, so every edge passes the filter and ties go
    # to the smaller index).  While all are Undecided, 0 votes for 1, 1 for 0,
    # 2 for 1, 3 for 2 and 4 for 3: votes grow by (1, 2, 1, 1, 0) per iteration,
    # so after iteration 4 vertex 1 has 8 votes and becomes a Seed.  Iteration 5:
    # 0 and 2 join Seed 1; 3 votes for 2 (still Undecided at the iteration's
    # start), 4 for 3.  Iterations 6-8: 3 and 4 vote for each other, 3 reaches 8
    # votes after iteration 8 and becomes a Seed; 4 joins it in iteration 9.
    # Final votes (4, 8, 5, 8, 3), aggregates {0, 1, 2} and {3, 4}.
    g = gg.path(5)
    nc, agg, state, idx, votes = oracle.aggregate(g, _uniform_S(g), oracle.default_opts())
    assert nc == 2
    assert list(agg) == [0, 0, 0, 1, 1]
    assert list(state) == [0, 2, 0, 2, 0]
    assert list(idx) == [1, 1, 1, 3, 3]
    assert list(votes) == [4, 8, 5, 8, 3]


def test_adjacent_roots_are_allowed():
    # two stars K_{1,9} whose hubs 0 and 10 are joined
    u = [0] * 9 + [10] * 9 + [0]
    v = list(range(1, 10)) + list(range(11, 20)) + [10]
    g = gg.from_edges(20, u, v)
    nc, agg, state, idx, votes = oracle.aggregate(g, _uniform_S(g), oracle.default_opts())
    assert nc == 2
    assert state[0] == 2 and state[10] == 2
    assert all(idx[1:10] == 0) and all(idx[11:20] == 10)


def test_aggregation_invariants_on_random_graphs():
    for mk in SMALL_GRAPHS:
        g = mk()
        _, S = oracle.soc(g)
        nc, agg, state, idx, votes = oracle.aggregate(g, S)
        roots = np.nonzero(idx == np.arange(g.n))[0]
        assert nc == roots.size
        assert np.array_equal(agg[roots], np.arange(nc))  # renumbered in increasing root id
        assert np.all(idx[idx] == idx)  # every index names a root
        assert np.array_equal(agg, agg[idx])
        for i in np.nonzero(idx != np.arange(g.n))[0]:
            assert idx[i] in g.col[g.row_ptr[i]:g.row_ptr[i + 1]]  # joined a neighbour
            assert state[idx[i]] == 2 and state[i] == 0


# -------------------------------------------------------------- Galerkin

def test_galerkin_matches_dense_triple_product():
    rng = np.random.default_rng(5)
    for mk in SMALL_GRAPHS:
        g = mk()
        nc = max(2, g.n // 4)
        agg = rng.integers(0, nc, g.n)
        agg[:nc] = np.arange(nc)  # every aggregate non-empty
        gc, cd = oracle.galerkin(g, agg, nc)
        R = np.zeros((nc, g.n))
        R[agg, np.arange(g.n)] = 1.0
        ref = R @ dense_L(g) @ R.T
        Lc = dense_L(gc, cd)
        assert np.abs(Lc - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.all(gc.w > 0)
        assert abs(Lc.sum()) <= 1e-12 * np.abs(ref).max() * nc
        rows = np.repeat(np.arange(g.n), g.degrees())
        inter = agg[rows] != agg[g.col]
        assert math.isclose(math.fsum(gc.w), math.fsum(g.w[inter]), rel_tol=1e-14)


# --------------------------------------------------- hierarchy invariants

def _check_laplacian_level(g, d):
    assert oracle.validate(g) in (0,)
    for i in range(g.n):
        row = g.w[g.row_ptr[i]:g.row_ptr[i + 1]]
        s = math.fsum(row)
        assert abs(d[i] - s) <= 0.5 * math.ulp(d[i]) + 0.0


@pytest.mark.parametrize("mk", [lambda: gg.grid2d(64, 64), lambda: gg.rmat(11, 16, seed=2),
                                lambda: gg.chung_lu(5000, seed=6, max_deg=300),
                                lambda: gg.grid3d(10, 10, 10, weights="loguniform", seed=4)])
def test_every_level_is_a_connected_laplacian(mk):
    g = mk()
    h = oracle.Hierarchy(g)
    levels = h.levels()
    assert levels[-1].type == oracle.COARSEST
    assert levels[-1].n + levels[-1].nnz <= 1000
    for l, L in enumerate(levels):
        gl, d = h.csr(l)
        _check_laplacian_level(gl, d)
        if l + 1 < len(levels):
            assert levels[l + 1].n == L.nc
            assert levels[l + 1].n < L.n
        if L.type == oracle.ELIM:
            assert l + 1 < len(levels) and levels[l + 1].type != oracle.ELIM


def test_coarsest_pseudo_inverse():
    g = gg.grid2d(20, 20)
    h = oracle.Hierarchy(g)
    gl, d = h.csr(h.num_levels - 1)
    L = dense_L(gl, d)
    P = h.coarsest_pinv()
    ref = np.linalg.pinv(L)
    assert np.abs(P - ref).max() <= 1e-9 * np.abs(ref).max()
    assert np.abs(L @ P @ L - L).max() <= 1e-10 * np.abs(L).max()


@pytest.mark.parametrize("scale", [1e-3, 1.0, 1e5])
def test_coarsest_pseudo_inverse_at_any_weight_scale(scale):
    """The dense direct solve stays accurate to rounding when the weights are
    far from 1: the null-space shift follows the diagonal's scale, so the
    inverted matrix is as well conditioned as L on the mean-zero space."""
    g = gg.gnp(60, 0.15, seed=5)
    g.w = g.w * scale
    d = np.bincount(np.repeat(np.arange(g.n), np.diff(g.row_ptr)), weights=g.w, minlength=g.n)
    P = oracle.pinv_dense(g)
    ref = np.linalg.pinv(dense_L(g, d))
    assert np.abs(P - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------------------------- eigenvalue

def test_tridiag_max_matches_eigvalsh():
    rng = np.random.default_rng(7)
    for m in range(1, 12):
        a = rng.standard_normal(m)
        b = rng.standard_normal(max(m - 1, 0))
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        assert math.isclose(oracle.tridiag_max(a, b), np.linalg.eigvalsh(T).max(), rel_tol=1e-12,
                            abs_tol=1e-12)


def test_lanczos_on_even_cycle_finds_two():
    g = gg.cycle(8)  # D^-1 L has eigenvalues 1 - cos(2 pi k / 8); the largest is 2
    lm = oracle.lanczos_lmax(g, steps=10)
    assert abs(lm - 2.0) < 1e-10


def test_lanczos_estimate_on_bipartite_grid():
    g = gg.grid2d(12, 12)  # bipartite: lambda_max(D^-1 L) = 2 exactly
    lm = oracle.lanczos_lmax(g, steps=10)
    assert 1.8 < lm <= 2.0 + 1e-12


def test_lanczos_estimate_does_not_depend_on_summation_order():
    """lambda_max is a stored hierarchy value, so its sums are exact: a level
    with every row's entries in another order gives the same bits.  The
    levels of a 65,536-vertex Chung-Lu hierarchy are sensitive enough that
    plain fp64 sums change the estimate's last bits under such a shuffle (the
    coarse level 3 by 7e-16)."""
    g = gg.chung_lu(1 << 16, seed=6)
    ho = oracle.Hierarchy(g)
    rng = np.random.default_rng(2)
    checked = 0
    for l, L in enumerate(ho.levels()):
        if L.type != oracle.AGG:
            continue
        G, d = ho.csr(l)
        col, w = G.col.copy(), G.w.copy()
        for i in range(G.n):
            a, b = G.row_ptr[i], G.row_ptr[i + 1]
            p = a + rng.permutation(b - a)
            col[a:b], w[a:b] = G.col[p], G.w[p]
        shuffled = gg.Graph(G.n, G.row_ptr, col, w)
        lm = oracle.lanczos_lmax(G, steps=10, level=l, d=d)
        assert lm == L.lmax
        assert oracle.lanczos_lmax(shuffled, steps=10, level=l, d=d) == lm, l
        if G.n <= 2000:  # and it is an estimate from below of the true lambda_max
            rows = np.repeat(np.arange(G.n), np.diff(G.row_ptr))
            Ld = np.zeros((G.n, G.n))
            Ld[rows, G.col] = -G.w
            Ld[np.arange(G.n), np.arange(G.n)] = d
            true = np.linalg.eigvals(Ld / d[:, None]).real.max()
            assert 0.8 * true < lm <= true * (1 + 1e-12), (l, lm, true)
        checked += 1
    assert checked >= 2


# -------------------------------------------------------------- smoother

def test_chebyshev_damps_eigenvectors_by_the_chebyshev_ratio():
    n = 16
    g = gg.cycle(n)  # D = 2I; D^-1 L u_k = mu_k u_k, mu_k = 1 - cos(2 pi k / n)
    opts = oracle.default_opts()
    lmax = 2.0
    lo, hi = opts.cheb_lo * lmax, opts.cheb_hi * lmax
    theta, delta = (hi + lo) / 2, (hi - lo) / 2

    def T2(t):
        return 2 * t * t - 1

    L = dense_L(g)
    i = np.arange(n)
    for k in range(n // 2 + 1):
        u = np.cos(2 * np.pi * k * i / n)
        mu = 1 - np.cos(2 * np.pi * k / n)
        b = L @ u
        x = oracle.cheb_apply(g, lmax, np.zeros(n), b, opts, x_is_zero=True)
        factor = T2((theta - mu) / delta) / T2(theta / delta)
        assert np.abs((u - x) - factor * u).max() <= 1e-13
        # from a non-zero start the error obeys the same polynomial
        x0 = 0.25 * u
        x = oracle.cheb_apply(g, lmax, x0, b, opts)
        assert np.abs((u - x) - factor * 0.75 * u).max() <= 1e-13


# ----------------------------------------------------------------- solve

SOLVE_GRAPHS = [
    lambda: gg.grid2d(15, 15),
    lambda: gg.gnp(200, 0.03, seed=4),
    lambda: gg.star(40),
    lambda: gg.path(60),
    lambda: gg.chung_lu(300, seed=4, max_deg=40),
    lambda: gg.grid3d(6, 6, 6, weights="loguniform", seed=8),
]


@pytest.mark.parametrize("cycle", [1, 2])
@pytest.mark.parametrize("mk", SOLVE_GRAPHS)
def test_solve_matches_dense_pseudo_inverse(mk, cycle):
    g = mk()
    h = oracle.Hierarchy(g, oracle.default_opts(cycle=cycle, coarsest_nnz=60))
    rng = np.random.default_rng(1)
    b = rng.standard_normal(g.n)
    x, st, it, rel, work = h.solve(b, 1e-8, 300)
    assert st == 0 and rel <= 1e-8
    L = dense_L(g)
    bp = b - b.mean()
    ref = np.linalg.pinv(L) @ bp
    ev = np.linalg.eigvalsh(L)
    lam1 = ev[1]
    # ||x - x*|| <= ||r|| / lambda_1 (both mean-zero)
    bound = 1.5 * rel * np.linalg.norm(bp) / lam1 + 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(x - ref) <= bound
    assert abs(x.mean()) < 1e-12 * (np.abs(x).max() + 1)
    assert np.linalg.norm(bp - L @ x) <= 1e-8 * np.linalg.norm(bp) * 1.0001


def test_solve_eigenvector_rhs_on_path():
    n = 50
    g = gg.path(n)
    h = oracle.Hierarchy(g, oracle.default_opts(coarsest_nnz=20))
    i = np.arange(n)
    for k in (1, 7, 30):
        u = np.cos(np.pi * k * (i + 0.5) / n)  # Laplacian eigenvector of the path
        lam = 2 - 2 * np.cos(np.pi * k / n)
        x, st, it, rel, work = h.solve(u, 1e-10, 200)
        assert st == 0
        assert np.linalg.norm(x - u / lam) <= 1e-8 * np.linalg.norm(u / lam) / (lam / 4.0)


def test_elimination_level_with_exact_coarse_solve_is_exact():
    g = gg.grid2d(10, 10)
    h = oracle.Hierarchy(g, oracle.default_opts(max_levels=2, coarsest_nnz=100))
    lv = h.levels()
    assert [L.type for L in lv] == [oracle.ELIM, oracle.COARSEST]
    rng = np.random.default_rng(2)
    b = rng.standard_normal(g.n)
    b -= b.mean()
    x = h.cycle(b)
    L = dense_L(g)
    assert np.linalg.norm(L @ x - b) <= 1e-12 * np.linalg.norm(b)
    x, st, it, rel, work = h.solve(b, 1e-8)
    assert st == 0 and it == 1


def test_repeated_elimination_keeps_series_resistance_on_a_path():
    # Eliminating vertices of a unit-weight path only deletes leaves or merges
    # series edges: a coarse edge between the surviving original vertices u < v
    # has weight 1/(v - u), the series resistance of the fine edges between them.
    n = 257
    g = gg.path(n)
    h = oracle.Hierarchy(g, oracle.default_opts(elim_passes=6, elim_min_fraction=0.0,
                                                coarsest_nnz=3))
    lv = h.levels()
    elim = [l for l, L in enumerate(lv) if L.type == oracle.ELIM]
    assert elim[:6] == list(range(6)), [L.type for L in lv]
    sizes = [lv[l].n for l in range(7)]
    assert all(a > b for a, b in zip(sizes, sizes[1:]))
    orig = np.arange(n)
    for l in range(6):  # original vertex behind each kept vertex
        cidx = h.map(l)
        kept = np.flatnonzero(cidx >= 0)
        new = np.empty(lv[l].nc, dtype=np.int64)
        new[cidx[kept]] = orig[kept]
        orig = new
    assert np.all(np.diff(orig) > 0)
    gc, dc = h.csr(6)
    rows = np.repeat(np.arange(gc.n), np.diff(gc.row_ptr))
    assert np.all(np.diff(gc.row_ptr) <= 2)  # still a path, between consecutive survivors
    assert np.all(np.abs(rows - gc.col) == 1)
    span = np.abs(orig[rows] - orig[gc.col]).astype(np.float64)
    assert np.allclose(gc.w * span, 1.0, rtol=1e-12, atol=0)


def test_repeated_elimination_with_exact_coarse_solve_is_exact():
    # elimination levels are exact Schur complements: with passes repeated
    # until the dense coarsest level, one cycle is L^+ and CG stops after one step
    g = gg.path(60, w=np.linspace(1.0, 3.0, 59))
    h = oracle.Hierarchy(g, oracle.default_opts(elim_passes=16, coarsest_nnz=60))
    lv = h.levels()
    assert [L.type for L in lv[:-1]] == [oracle.ELIM] * (len(lv) - 1) and len(lv) >= 3
    rng = np.random.default_rng(5)
    b = rng.standard_normal(g.n)
    b -= b.mean()
    L = dense_L(g)
    x = h.cycle(b)
    assert np.linalg.norm(L @ x - b) <= 1e-12 * np.linalg.norm(b)
    x, st, it, rel, work = h.solve(b, 1e-8)
    assert st == 0 and it == 1


def test_wda_within_the_papers_range_on_the_2d_grid():
    # context only: the paper's V-cycle WDA on its test set spans roughly 3 to 100
    g = gg.grid2d(64, 64)
    h = oracle.Hierarchy(g)
    b = gg.rhs(g.n, 1, 1)[:, 0]
    x, st, it, rel, work = h.solve(b)
    wda = -work / math.log10(rel)
    assert st == 0 and 3 < wda < 100


# ---- eigenpairs (the definition computed densely; pinned to closed forms)
def test_eigs_dense_path_closed_form_and_fiedler_vector():
    n = 40
    lam, V = oracle.eigs_dense(gg.path(n), 3)
    k = np.arange(1, 4)
    assert np.allclose(lam, 2.0 - 2.0 * np.cos(np.pi * k / n), rtol=0, atol=1e-12)
    u = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    assert abs(abs(V[:, 0] @ u) / np.linalg.norm(u) - 1.0) <= 1e-10


def test_eigs_dense_even_cycle_has_double_eigenvalues():
    n = 30
    lam, V = oracle.eigs_dense(gg.cycle(n), 4)
    want = 2.0 - 2.0 * np.cos(2.0 * np.pi * np.array([1, 1, 2, 2]) / n)
    assert np.allclose(lam, want, rtol=0, atol=1e-12)


def test_eigs_dense_grid_is_a_sum_of_path_spectra():
    a, b = 7, 5
    lam, V = oracle.eigs_dense(gg.grid2d(a, b), 6)
    pa = 2.0 - 2.0 * np.cos(np.pi * np.arange(a) / a)
    pb = 2.0 - 2.0 * np.cos(np.pi * np.arange(b) / b)
    want = np.sort((pa[:, None] + pb[None, :]).ravel())[1:7]
    assert np.allclose(lam, want, rtol=0, atol=1e-12)
    assert np.allclose(V.T @ V, np.eye(6), atol=1e-12)
    assert np.allclose(V.sum(axis=0), 0.0, atol=1e-10)  # orthogonal to the constant


@pytest.mark.parametrize("mk", [lambda: gg.grid2d(64, 64), lambda: gg.rmat(11, 16, seed=2),
                                lambda: gg.grid3d(9, 8, 7, weights="loguniform", seed=4)])
def test_laplacian_product_matches_scipy_on_every_level(mk):
    """The oracle's L x (Section 2.1, L = D - A) on every level of a hierarchy,
    against scipy's sparse product with the level's own diagonal; and L 1 = 0
    up to the rounding of the row sums."""
    g = mk()
    h = oracle.Hierarchy(g)
    rng = np.random.default_rng(21)
    for l in range(h.num_levels):
        gl, d = h.csr(l)
        A = sparse_A(gl)
        x = rng.standard_normal(gl.n)
        y = h.spmv(l, x)
        ref = d * x - A @ x
        scale = d * np.abs(x) + abs(A) @ np.abs(x)
        assert np.all(np.abs(y - ref) <= 1e-13 * scale + 1e-300), l
        y1 = h.spmv(l, np.ones(gl.n))
        assert np.all(np.abs(y1) <= 1e-13 * d + 1e-300), l
        # a planted sign error (L = D + A) would fail the first check
        assert gl.nnz == 0 or not np.allclose(d * x + A @ x, ref)


# ---------------------------------------------- K-cycle inner solve (3.7)

def _fcg_levels(h):
    """Levels whose coarse solve is the K-cycle's inner FCG: the coarse level
    of an aggregation level, unless it is the coarsest."""
    lv = h.levels()
    return [l for l in range(1, len(lv))
            if lv[l - 1].type == oracle.AGG and lv[l].type != oracle.COARSEST]


@pytest.mark.parametrize("cycle", [1, 2])
@pytest.mark.parametrize("mk", [lambda: gg.grid2d(40, 40),
                                lambda: gg.chung_lu(4000, seed=9, max_deg=300),
                                lambda: gg.grid3d(10, 10, 10, weights="loguniform", seed=2)])
def test_kcycle_inner_fcg_minimises_energy_over_its_two_directions(mk, cycle):
    """Two steps of flexible CG from x = 0 with preconditioner M (the cycle
    from that level) give the L-energy minimiser of the error over the span
    of p1 = M b and M r1, r1 = b - a1 L p1 (the second direction differs from
    M r1 by a multiple of p1 only).  Equivalently the residual b - L x is
    orthogonal to both directions (Galerkin condition).  The reference here
    is that minimiser from a dense 2x2 solve with scipy's L; a wrong sign of
    the orthogonalisation coefficient, or a skipped orthogonalisation, moves
    x off it."""
    g = mk()
    h = oracle.Hierarchy(g, oracle.default_opts(cycle=cycle))
    targets = _fcg_levels(h)
    assert targets, "hierarchy has no level with an inner FCG"
    rng = np.random.default_rng(5)
    for l in targets:
        G, d = h.csr(l)
        L = (sp.diags(d) - sparse_A(G)).tocsr()
        b = rng.standard_normal(G.n)
        b -= b.mean()
        x = h.level_fcg2(l, b)
        p1 = h.level_cycle(l, b)
        q1 = L @ p1
        r1 = b - (p1 @ b) / (p1 @ q1) * q1
        V = np.stack([p1, h.level_cycle(l, r1)], axis=1)
        xs = V @ np.linalg.solve(V.T @ (L @ V), V.T @ b)
        e = x - xs
        err = math.sqrt(max(e @ (L @ e), 0.0)) / math.sqrt(xs @ (L @ xs))
        assert err <= 1e-9, (l, err)
        r = b - L @ x
        for v in V.T:
            assert abs(v @ r) <= 1e-9 * np.linalg.norm(v) * np.linalg.norm(b), l


# --------------------------------------------------- work count (2.3.1)
# Work is counted in units of one finest-level residual, i.e. nnz(L_0) =
# n_0 + nnz(A_0) multiply-adds, and every operator application adds the
# nonzeros of that operator (Section 2.3.1).  With Chebyshev degree 2: an
# aggregation level costs 1 L (pre-smoothing from zero: its first step needs
# no product) + 1 L (residual) + n (R) + n (P) + 2 L (post-smoothing) plus its
# coarse solve; an elimination level costs nnz(P) (restriction P^T) + nnz(P)
# + |F| (prolongation and the F-point update) plus its coarse solve; the
# coarsest level costs n_c^2 (dense L^+).  The totals below are counted by
# hand from those rules on hierarchies whose structure is asserted first.

def _structure(h):
    return [(L.type, L.n, L.nnz, L.nc) for L in h.levels()]


def test_cycle_work_hand_count_star():
    # K_{1,9} without elimination, coarsest at n + nnz <= 10: the nine leaves
    # vote for the hub, so one aggregate.  nnz(L_0) = 10 + 18 = 28.
    # Level 0: 28 + 28 + 10 + 10 + 2 * 28 = 132; coarsest 1^2 = 1.
    h = oracle.Hierarchy(gg.star(9), oracle.default_opts(elim_enable=0, coarsest_nnz=10))
    assert _structure(h) == [(oracle.AGG, 10, 18, 1), (oracle.COARSEST, 1, 0, 0)]
    assert h.cycle_work() == pytest.approx(133 / 28, rel=1e-15)


def test_cycle_work_hand_count_elimination():
    # Path 0-1-2-3-4 with the identity hash: only vertex 0 is a local minimum,
    # so F = {0}, C = {1, 2, 3, 4}; nnz(P) = |C| + deg(0) = 4 + 1 = 5.
    # Level 0: 5 (P^T) + 5 (P) + 1 (F update) = 11; coarsest path of 4 vertices:
    # 4^2 = 16.  nnz(L_0) = 5 + 8 = 13.
    h = oracle.Hierarchy(gg.path(5), oracle.default_opts(hash_mode=1, coarsest_nnz=10))
    assert _structure(h) == [(oracle.ELIM, 5, 8, 4), (oracle.COARSEST, 4, 6, 0)]
    assert h.cycle_work() == pytest.approx(27 / 13, rel=1e-15)


def test_cycle_work_hand_count_v_and_k_cycles():
    # Path of 7 without elimination, coarsest at n + nnz <= 6:
    # aggregation 7 -> 3 -> coarsest 1.  nnz(L_0) = 19, nnz(L_1) = 7.
    # V: level 1 = 7 + 7 + 3 + 3 + 14 = 34, coarsest 1, level 0 = 19 + 19 + 7
    #    + 7 + 38 = 90 plus 35 -> 125.
    # K: level 0's coarse solve is two FCG steps on level 1, each one cycle
    #    from level 1 (35) and one product with L_1 (7): 84 -> 90 + 84 = 174.
    for cycle, units in ((1, 125), (2, 174)):
        h = oracle.Hierarchy(gg.path(7), oracle.default_opts(elim_enable=0, coarsest_nnz=6,
                                                             cycle=cycle))
        assert _structure(h) == [(oracle.AGG, 7, 12, 3), (oracle.AGG, 3, 4, 1),
                                 (oracle.COARSEST, 1, 0, 0)]
        assert h.cycle_work() == pytest.approx(units / 19, rel=1e-15), cycle


def test_solve_work_counts_cycles_and_products():
    # PCG (Section 2.3.2) applies the cycle once before the loop and once per
    # further iteration, one product with L_0 per iteration, and one more for
    # the true residual that confirms convergence: it * (cycle + 1) + 1 units
    # when no restart happens (the solve below converges without one).
    g = gg.path(7)
    h = oracle.Hierarchy(g, oracle.default_opts(elim_enable=0, coarsest_nnz=6))
    b = np.linspace(-1.0, 1.0, g.n) ** 3
    x, st, it, rel, work = h.solve(b, 1e-10, 50)
    assert st == 0 and it >= 2
    assert work == pytest.approx(it * (125 / 19 + 1) + 1, rel=1e-14)
