"""Host-side behaviour of bench.py: the one-GPU guard and the HBM traffic
figures it takes from committed counter summaries (keyed by a hash of the
kernel sources, so a changed kernel reports no stale traffic)."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    for extra, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + extra,
                           capture_output=True, text=True, timeout=120,
                           env=dict(os.environ, **env))
        assert r.returncode == 2
        assert "one GPU only" in r.stderr


def _write_summary(dirpath, family, workload, source_hash, nbytes):
    rec = {"workload": workload, "family": family, "kernel_source_hash": source_hash,
           "hbm_bytes_per_launch": nbytes}
    path = os.path.join(dirpath, f"{family}_{workload}_pmc.txt")
    with open(path, "w") as f:
        f.write("# summary\n\njson: " + json.dumps(rec) + "\n")


def test_traffic_is_taken_only_from_summaries_of_the_current_kernels(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    current = bench.kernel_source_hash()
    assert len(current) == 16
    assert bench.load_traffic("spmv", "rmat_s18") is None  # no summary
    _write_summary(tmp_path, "spmv", "rmat_s18", current, 1.25e8)
    assert bench.load_traffic("spmv", "rmat_s18") == 1.25e8
    _write_summary(tmp_path, "spmv", "rmat_s18", "0" * 16, 1.25e8)
    assert bench.load_traffic("spmv", "rmat_s18") is None  # taken on other kernels


def test_every_workload_names_a_graph_recipe():
    import graphgen as gg

    for name, wl in bench.WORKLOADS.items():
        assert wl["cfg"] in gg.CONFIGS, name
        assert set(wl["family"].split(",")) <= {"spmv", "lanczos", "cheb", "cheb0", "cheb1", "resid", "resid64", "cg_update"}, name


def test_cpu_baseline_times_setup_and_solves_apart():
    import graphgen as gg

    g = gg.grid2d(24, 24)
    B = gg.rhs(g.n, 2, 1)
    full = bench.cpu_baseline(g, B, k=2, iters=1000)
    assert full["kind"] == "oracle" and full["cores"] >= 1 and full["value"] > 0
    assert full["setup_s"] > 0 and full["solve_s_per_rhs"] > 0
    assert "solved to 1e-8" in full["sample"]
    assert full["host"]["nproc"] >= 1
    # a solve longer than the sample cap is timed for that many iterations and scaled
    part = bench.cpu_baseline(g, B, k=2, iters=40, max_sample_iters=5)
    assert "5 CG iterations" in part["sample"] and part["iters"] == 40


def test_roofline_kernels_are_matched_at_every_unroll():
    """rocprofv3 names a column-split kernel with its unroll argument; the
    roofline kernel counts its instances at every unroll together."""
    col = "void lg::k_rows_col<lg::LapColOp<double, 16, 1, 0>, 4>(lg::LapColOp<double, 16, 1, 0>, int const*)"
    assert bench._kernel_of(col) == "k_rows_col<lg::LapColOp<double, 16, 1, 0> >"
    assert bench._kernel_of(col.replace(", 4>(", ", 6>(")) == bench._kernel_of(col)
    one = "void lg::k_rows<lg::LapOp<double, 1, 1, 0> >(lg::LapOp<double, 1, 1, 0>, int const*)"
    assert bench._kernel_of(one) == "k_rows<lg::LapOp<double, 1, 1, 0> >"
    names = {w["kernel"] for w in bench.WORKLOADS.values()}
    assert all(not bench._UNROLL_ARG.match(n) for n in names)
