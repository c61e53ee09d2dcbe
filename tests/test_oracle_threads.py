"""The OpenMP build of the oracle (used only to time the CPU baseline) computes
the same bits as the single-threaded build the tests pin: only loops whose
iterations write their own rows run in parallel."""

import numpy as np
import pytest

import graphgen as gg
import oracle


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("mk", [lambda: gg.chung_lu(20000, seed=6, max_deg=2000),
                                lambda: gg.grid3d(14, 14, 14, weights="loguniform", seed=4),
                                lambda: gg.rmat(12, 16, seed=2)])
@pytest.mark.parametrize("cycle", [1, 2])
def test_threaded_oracle_is_bit_identical(mk, cycle):
    g = mk()
    opts = oracle.default_opts(cycle=cycle)
    h1 = oracle.Hierarchy(g, opts)
    h2 = oracle.Hierarchy(g, oracle.default_opts(cycle=cycle), threaded=True)
    assert oracle.threads(True) >= 1
    L1, L2 = h1.levels(), h2.levels()
    assert [(L.type, L.n, L.nnz, L.nc) for L in L1] == [(L.type, L.n, L.nnz, L.nc) for L in L2]
    for l, L in enumerate(L1):
        assert _bits([L.lmax]) == _bits([L2[l].lmax])
        (a, da), (b, db) = h1.csr(l), h2.csr(l)
        assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
        assert np.array_equal(_bits(a.w), _bits(b.w)) and np.array_equal(_bits(da), _bits(db))
        if L.type == oracle.COARSEST:
            continue
        assert np.array_equal(h1.map(l), h2.map(l))
        if L.type == oracle.AGG:
            X1, S1 = h1.soc(l)
            X2, S2 = h2.soc(l)
            assert np.array_equal(_bits(X1), _bits(X2)) and np.array_equal(_bits(S1), _bits(S2))
            for u, v in zip(h1.votes(l), h2.votes(l)):
                assert np.array_equal(u, v)
        else:
            assert np.array_equal(h1.elim_z(l), h2.elim_z(l))
    assert np.array_equal(_bits(h1.coarsest_pinv()), _bits(h2.coarsest_pinv()))
    b = gg.rhs(g.n, 1, 4)[:, 0]
    x1, s1, i1, r1, w1 = h1.solve(b, 1e-8, 300)
    x2, s2, i2, r2, w2 = h2.solve(b, 1e-8, 300)
    assert (s1, i1) == (s2, i2) and _bits([r1, w1]).tolist() == _bits([r2, w2]).tolist()
    assert np.array_equal(_bits(x1), _bits(x2))
