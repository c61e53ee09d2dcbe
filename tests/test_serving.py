"""The continuous-batching solve server (lg_server_*): every request's result
is the same alone and in the mix and agrees with the CPU oracle (within the
solver's stated tolerance; bit for bit at equal batch width), requests join a
running session as slots free up, hierarchies are admitted by the HBM budget,
and a bad graph fails only its own requests.  All calls go through the C ABI.
"""

import time

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1705_06266_amd.lgmg as lg
from gpu_util import dense_laplacian_norm, laplacian_apply, oracle_opts, say, to_dev

pytestmark = pytest.mark.gpu

POOL = [
    lambda: gg.grid2d(40, 40),
    lambda: gg.rmat(11, 16, seed=5),
    lambda: gg.chung_lu(5000, seed=8, max_deg=800),
    lambda: gg.grid3d(10, 10, 10, weights="loguniform", seed=9),
    lambda: gg.path(600),
    lambda: gg.gnp(800, 0.01, seed=10),
    # level 0 stored in the solve-time vertex order
    lambda: gg.chung_lu(30000, mean_deg=48, max_deg=5000, seed=11),
]


def _requests(graphs, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        gid = i % len(graphs)
        k = int(rng.integers(1, 9))
        out.append((gid, gg.rhs(graphs[gid].n, k, 100 + i)))
    return out


def _same_within_tolerance(g, b, X, infos, Xa, infa):
    """Both solve L x = b to 1e-8: energy-norm difference <= 1e-6 (the bar of
    the fp64 parity tests), iteration counts within one."""
    for c in range(b.shape[1]):
        bp = b[:, c] - b[:, c].mean()
        rel = np.linalg.norm(bp - laplacian_apply(g, X[:, c])) / np.linalg.norm(bp)
        assert rel <= 1e-8 * 1.001
        diff = dense_laplacian_norm(g, X[:, c] - Xa[:, c]) / dense_laplacian_norm(g, Xa[:, c])
        assert diff <= 1e-6, (c, diff)
        assert abs(infos[c]["iters"] - infa[c]["iters"]) <= 1


def _matches_oracle(g, ho, b, X, infos):
    """Each column against the oracle's FP64 solve of the same right-hand side:
    energy-norm difference <= 1e-6, iteration counts within one."""
    for c in range(b.shape[1]):
        xo, sto, ito, relo, _ = ho.solve(b[:, c], 1e-8, 500)
        assert sto == 0
        diff = dense_laplacian_norm(g, X[:, c] - xo) / dense_laplacian_norm(g, xo)
        assert diff <= 1e-6, (c, diff)
        assert abs(infos[c]["iters"] - ito) <= 1, (c, infos[c]["iters"], ito)


def _alone(graphs, max_batch_rhs):
    """One hierarchy per graph built like the server's (max_rhs = max_batch_rhs)."""
    return [lg.lg_setup(g.row_ptr, g.col, g.w, lg.lg_default_opts(max_rhs=max_batch_rhs))
            for g in graphs]


@pytest.fixture(scope="module")
def graphs():
    import torch

    assert torch.cuda.is_available()
    return [mk() for mk in POOL]


def test_results_are_the_same_alone_and_in_the_mix(graphs):
    import torch

    reqs = _requests(graphs, 36, 1)
    srv = lg.Server(workers=3, max_batch_rhs=32)
    gids = [srv.add_graph(g.row_ptr, g.col, g.w) for g in graphs]
    dev = [to_dev(b) for _, b in reqs]
    torch.cuda.synchronize()  # inputs final before the server's streams read them
    ids = [srv.submit(gids[gid], B) for (gid, _), B in zip(reqs, dev)]
    results = [srv.wait(i) for i in ids]
    st = srv.stats()
    say(f"  server stats {st}")
    srv.close()
    assert st["completed"] == len(reqs) and st["setups"] == len(graphs)
    assert st["batches"] < len(reqs), "requests on one graph should share batches"
    alone = _alone(graphs, 32)
    ho = [oracle.Hierarchy(g, oracle_opts(lg.lg_default_opts())) for g in graphs]
    for (gid, b), (X, infos, status, lat) in zip(reqs, results):
        Xa, infa, sta = lg.lg_solve(alone[gid], to_dev(b))
        assert status == lg.LG_OK and sta == lg.LG_OK and lat > 0.0
        _same_within_tolerance(graphs[gid], b, X.cpu().numpy(), infos, Xa.cpu().numpy(), infa)
        _matches_oracle(graphs[gid], ho[gid], b, X.cpu().numpy(), infos)


def test_requests_join_a_running_session(graphs):
    """Slot-level admission: with one worker, requests on a graph submitted
    while a session on it runs enter that session's free slots at an iteration
    boundary (no new session), and every result matches the oracle."""
    import torch

    g = gg.grid3d(16, 16, 16, weights="loguniform", seed=12)  # a few hundred CG iterations
    srv = lg.Server(workers=1, max_batch_rhs=8)
    gid = srv.add_graph(g.row_ptr, g.col, g.w)
    warm = to_dev(gg.rhs(g.n, 1, 40))
    torch.cuda.synchronize()
    srv.wait(srv.submit(gid, warm))  # builds the hierarchy
    before = srv.stats()
    first = gg.rhs(g.n, 5, 41)  # a session of width 8: three idle slots
    later = [gg.rhs(g.n, 1, 42 + i) for i in range(3)]
    dev = [to_dev(first)] + [to_dev(b) for b in later]
    torch.cuda.synchronize()
    rid = [srv.submit(gid, dev[0])]
    time.sleep(0.005)
    for B in dev[1:]:
        rid.append(srv.submit(gid, B))
        time.sleep(0.002)
    results = [srv.wait(r) for r in rid]
    after = srv.stats()
    srv.close()
    say(f"  stats before {before} after {after}")
    assert after["batches"] - before["batches"] == 1, "later requests should join the session"
    assert after["refills"] - before["refills"] == 3
    ho = oracle.Hierarchy(g, oracle_opts(lg.lg_default_opts()))
    for b, (X, infos, status, lat) in zip([first] + later, results):
        assert status == lg.LG_OK
        _matches_oracle(g, ho, b, X.cpu().numpy(), infos)


def test_admission_by_budget_evicts_idle_hierarchies(graphs):
    import torch

    reqs = _requests(graphs, 18, 2)
    srv = lg.Server(workers=2, max_batch_rhs=8, hbm_budget=1)  # no two hierarchies fit
    gids = [srv.add_graph(g.row_ptr, g.col, g.w) for g in graphs]
    dev = [to_dev(b) for _, b in reqs]
    torch.cuda.synchronize()  # inputs final before the server's streams read them
    ids = [srv.submit(gids[gid], B) for (gid, _), B in zip(reqs, dev)]
    results = [srv.wait(i) for i in ids]
    st = srv.stats()
    say(f"  server stats {st}")
    srv.close()
    assert st["evictions"] > 0 and st["resident_graphs"] <= 1
    alone = _alone(graphs, 8)
    for (gid, b), (X, infos, status, lat) in zip(reqs, results):
        Xa, infa, _ = lg.lg_solve(alone[gid], to_dev(b))
        assert status == lg.LG_OK
        _same_within_tolerance(graphs[gid], b, X.cpu().numpy(), infos, Xa.cpu().numpy(), infa)


def test_columns_of_a_batch_do_not_influence_each_other(graphs):
    """At one batch width, a column's result is bit-identical whatever the
    other columns hold (including a restart or an early convergence there)."""
    h = lg.lg_setup(graphs[2].row_ptr, graphs[2].col, graphs[2].w, lg.lg_default_opts(max_rhs=8))
    n = graphs[2].n
    A = gg.rhs(n, 3, 21)
    B1 = np.concatenate([A, gg.rhs(n, 2, 22)], axis=1)
    B2 = np.concatenate([A, np.zeros((n, 1)), 1e6 * gg.rhs(n, 1, 23)], axis=1)
    X1, i1, _ = lg.lg_solve(h, to_dev(B1))
    X2, i2, _ = lg.lg_solve(h, to_dev(B2))
    assert np.array_equal(X1.cpu().numpy()[:, :3], X2.cpu().numpy()[:, :3])
    assert [i["iters"] for i in i1[:3]] == [i["iters"] for i in i2[:3]]


def test_a_bad_graph_fails_only_its_requests(graphs):
    import torch

    two = gg.from_edges(6, [0, 1, 3, 4], [1, 2, 4, 5])  # two components
    srv = lg.Server(workers=2, max_batch_rhs=4)
    good = srv.add_graph(graphs[0].row_ptr, graphs[0].col, graphs[0].w)
    bad = srv.add_graph(two.row_ptr, two.col, two.w)
    Bb, Bg = to_dev(gg.rhs(two.n, 2, 1)), to_dev(gg.rhs(graphs[0].n, 3, 2))
    torch.cuda.synchronize()
    rb = srv.submit(bad, Bb)
    rg = srv.submit(good, Bg)
    with pytest.raises(lg.LgError) as e:
        srv.wait(rb)
    assert e.value.code == lg.LG_E_DISCONNECTED
    X, infos, status, lat = srv.wait(rg)
    assert status == lg.LG_OK and all(i["rel_residual"] <= 1e-8 for i in infos)
    with pytest.raises(lg.LgError) as e:
        srv.submit(good, to_dev(gg.rhs(graphs[0].n, 5, 3)))  # more than max_batch_rhs
    assert e.value.code == lg.LG_E_ARG
    srv.close()
