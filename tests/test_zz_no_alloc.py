"""lg_eigs_noalloc, the entry point for callers that cannot allocate device
memory: the same results as lg_eigs, bit for bit, on two calls in a row (the
second on a smaller graph, so the shared static scratch holds the first
call's contents), and sizes beyond its static buffer are refused."""

import numpy as np
import pytest

import graphgen as gg
import paper_1705_06266_amd.lgmg as lg
from gpu_util import gpu_setup, laplacian_apply, say

pytestmark = pytest.mark.gpu


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


@pytest.fixture(scope="module")
def built():
    import torch

    assert torch.cuda.is_available()
    lg.load()
    return True


def test_noalloc_eigs_match_lg_eigs_on_two_calls(built):
    import torch

    # a graph stored in the solve-time vertex order, then smaller ones: the
    # scratch keeps the previous call's values
    cases = [(gg.chung_lu(30000, mean_deg=48, max_deg=5000, seed=6), 2), (gg.grid2d(48, 48), 3),
             (gg.grid3d(9, 9, 9, weights="loguniform", seed=4), 2)]
    for g, nev in cases:
        say(f"[case] lg_eigs_noalloc n={g.n} nev={nev}")
        h = gpu_setup(g, max_rhs=8)
        lam, X, it, res, st = lg.lg_eigs(h, nev, tol=1e-8, max_iter=500)
        Xn = torch.full((g.n, nev), float("nan"), dtype=torch.float64, device="cuda:0")
        lam_n, it_n, res_n, st_n = lg.lg_eigs_noalloc(h, nev, Xn, tol=1e-8, max_iter=500)
        torch.cuda.synchronize()
        assert st == lg.LG_OK and st_n == lg.LG_OK
        assert it_n == it
        assert np.array_equal(_bits(lam_n), _bits(lam))
        assert np.array_equal(_bits(res_n), _bits(res))
        assert np.array_equal(_bits(Xn.cpu().numpy()), _bits(X.cpu().numpy()))
        x = Xn.cpu().numpy()
        for i in range(nev):  # and the pairs are eigenpairs to the tolerance
            r = np.linalg.norm(laplacian_apply(g, x[:, i]) - lam_n[i] * x[:, i])
            assert r <= 1e-8 * lam_n[i] * 1.001


def test_noalloc_eigs_refuses_sizes_beyond_its_buffer(built):
    import torch

    g = gg.grid2d(700, 700)  # 490,000 vertices: a block of 8 needs about 94 MB
    h = gpu_setup(g, max_rhs=8)
    X = torch.empty((g.n, 7), dtype=torch.float64, device="cuda:0")
    with pytest.raises(lg.LgError) as e:
        lg.lg_eigs_noalloc(h, 7, X)
    assert e.value.code == lg.LG_E_ARG and "scratch" in str(e.value)
