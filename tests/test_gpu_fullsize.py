"""Parity with the CPU oracle at the benchmark workloads' full sizes.

The small cases in test_gpu_parity.py fit in a few tiles of every setup
primitive.  These run the graphs the benchmark times, with the options it
times them with (precision, batch width, autotuner, graph replay), so that the
code paths that only large inputs reach are compared with the oracle too:

* scans over more than 1024 tiles of 2048 items (the recursive tile-sum
  branch): the nnz-sized count scans of R-MAT's elimination level (7.6M
  entries), the Galerkin emit scans of the 3D grid (12.5M) and the 1M-vertex
  Chung-Lu graph (15M);
* multi-tile radix passes of the Galerkin pair sort over millions of pairs;
* hub rows of degree up to 5.6e4, cut into thousands of chunks.

Bar, as in the small cases: every level (CSR, diagonal, transfer map), the
elimination product z, test vectors, strengths, voting state, roots and votes
bit for bit (Algorithms 2-3, Sections 3.4-3.5); one FP64 cycle to 1e-10 of
the oracle's; the benchmark's solve checked column by column with the true
residual recomputed on the host, and against the oracle's FP64 solve where the
oracle finishes in seconds (energy norm 1e-6 for FP64, 1e-5 for the mixed
form, the stated bound).

The 4M-vertex Chung-Lu workload (the benchmark's default, 63.9M nnz, largest
degree 6.9e4) runs in full, and the same generator at 2^20 vertices as a second
power-law case.  The oracle here is its OpenMP build, which computes the same
bits as the single-threaded one (test_oracle_threads.py) in a fraction of the
host time.
"""

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1705_06266_amd.lgmg as lg
from gpu_util import compare_hierarchies, dense_laplacian_norm, gpu_setup, oracle_opts, say, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]

# graph, right-hand sides (count, seed) and precision as the benchmark runs them
FULL = {
    "rmat_s18": dict(graph=lambda: gg.config_graph("rmat_s18"), k=1, seed=3,
                     precision=lg.LG_FP64, oracle_solve=True),
    "grid3d_128_loguniform": dict(graph=lambda: gg.config_graph("grid3d_128_loguniform"), k=32,
                                  seed=5, precision=lg.LG_MIXED, oracle_solve=False),
    "chunglu_1m": dict(graph=lambda: gg.chung_lu(1 << 20, seed=6), k=16, seed=6,
                       precision=lg.LG_MIXED, oracle_solve=True),
    "chunglu_4m": dict(graph=lambda: gg.config_graph("chunglu_4m"), k=16, seed=6,
                       precision=lg.LG_FP64, oracle_solve=True),
}


@pytest.fixture(scope="module")
def built():
    import torch

    assert torch.cuda.is_available()
    lg.load()
    return True


@pytest.fixture(scope="module", params=list(FULL))
def case(request, built):
    """(name, graph, oracle hierarchy); module scope, so pytest runs every test
    of one workload before building the next."""
    name = request.param
    g = FULL[name]["graph"]()
    say(f"[full] {name}: n={g.n} nnz={g.nnz} max degree={int(np.diff(g.row_ptr).max())}")
    ho = oracle.Hierarchy(g, oracle_opts(lg.lg_default_opts()), threaded=True)
    yield name, g, ho
    del ho


def _host_laplacian(g):
    import scipy.sparse as sp

    A = sp.csr_matrix((g.w, g.col, g.row_ptr), shape=(g.n, g.n))
    d = np.asarray(A.sum(axis=1)).ravel()
    return A, d


def test_fullsize_hierarchy_bit_exact(case):
    name, g, ho = case
    cfg = FULL[name]
    hg = gpu_setup(g, keep_setup_data=1, precision=cfg["precision"], max_rhs=cfg["k"])
    sg = compare_hierarchies(hg, ho, setup_data=True)
    say(f"  levels={[(s['type'], s['n'], s['nnz']) for s in sg]}")


def test_fullsize_fp64_cycle(case):
    """One FP64 cycle at the benchmark's width of 16 columns (column-split
    kernels, the fused coarse-correction step), two columns against the
    oracle's cycle."""
    name, g, ho = case
    hg = gpu_setup(g, max_rhs=16)
    B = gg.rhs(g.n, 16, 17)
    B -= B.mean(axis=0)
    X = lg.lg_cycle(hg, to_dev(B)).cpu().numpy()
    for c in (0, 15):
        xo = ho.cycle(B[:, c])
        err = np.linalg.norm(X[:, c] - xo) / np.linalg.norm(xo)
        say(f"  column {c}: relative difference {err:.2e}")
        assert err <= 1e-10


def test_fullsize_benchmark_solve(case):
    """The benchmark's own solve (its precision, width and right-hand sides)."""
    name, g, ho = case
    cfg = FULL[name]
    h = gpu_setup(g, precision=cfg["precision"], max_rhs=cfg["k"])
    B = gg.rhs(g.n, cfg["k"], cfg["seed"])
    X, info, st = lg.lg_solve(h, to_dev(B), rtol=1e-8, max_iter=500)
    assert st == 0
    X = X.cpu().numpy()
    A, d = _host_laplacian(g)
    Bp = B - B.mean(axis=0)
    R = Bp - (d[:, None] * X - A @ X)
    rel = np.linalg.norm(R, axis=0) / np.linalg.norm(Bp, axis=0)
    say(f"  iterations {[i['iters'] for i in info]}, worst true residual {rel.max():.2e}")
    assert np.all(rel <= 1e-8 * 1.001)
    for c in range(cfg["k"]):
        assert abs(info[c]["rel_residual"] - rel[c]) <= 1e-3 * rel[c] + 1e-13
    assert np.all(np.abs(X.mean(axis=0)) <= 1e-12 * np.abs(X).max(axis=0))
    if cfg["oracle_solve"]:
        xo, sto, ito, relo, _ = ho.solve(B[:, 0], 1e-8, 500)
        assert sto == 0
        diff = dense_laplacian_norm(g, X[:, 0] - xo) / dense_laplacian_norm(g, xo)
        say(f"  column 0: gpu iters {info[0]['iters']}, oracle {ito}, energy difference {diff:.1e}")
        assert diff <= (1e-6 if cfg["precision"] == lg.LG_FP64 else 1e-5)
        assert abs(info[0]["iters"] - ito) <= 1
