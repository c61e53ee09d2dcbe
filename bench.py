"""Benchmark: solves/s of the whole hot path on one MI355X.

One step = one pass of the whole path over one batch of input already in HBM:
setup (validation, elimination, strength of connection, voting aggregation,
Galerkin products, Lanczos, coarsest pseudo-inverse) followed by the solve of
the batch's right-hand sides to a 1e-8 relative residual.  The default
workload is the R-MAT scale-18 graph (edge factor 16, largest component,
U(0,1] weights) with one Gaussian right-hand side in FP64.

Prints one JSON line.  Besides the headline value it reports the solve-only
latency distribution on a resident hierarchy, the fp64 SpMV bandwidth of the
finest level, the dominant kernel against the HBM roofline (HIP events around
its launches inside the timed region) and the CPU oracle on a bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solves/s + p50/p99 latency to 1e-8 rel. residual; SpMV GB/s, mixed vs FP64"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1705_06266_amd/csrc/common.h", "paper_1705_06266_amd/csrc/ops.h",
                  "paper_1705_06266_amd/csrc/solve.hip", "paper_1705_06266_amd/csrc/setup.hip",
                  "paper_1705_06266_amd/csrc/prims.hip"]

WORKLOADS = {
    "rmat_s18": dict(cfg="c2_rmat_s18", precision="fp64", k=1,
                     label="rmat_s18_ef16_lcc_u01_fp64_1rhs"),
    "grid2d_64": dict(cfg="c1_grid2d_64", precision="fp64", k=1,
                      label="grid2d_64x64_unit_fp64_1rhs"),
    "grid3d_128_mixed": dict(cfg="c3_grid3d_128", precision="mixed", k=32,
                             label="grid3d_128cube_loguniform_mixed_32rhs"),
    "grid3d_128_fp64": dict(cfg="c3_grid3d_128", precision="fp64", k=32,
                            label="grid3d_128cube_loguniform_fp64_32rhs"),
    "chunglu_4m_mixed": dict(cfg="c4_chunglu_4m", precision="mixed", k=16,
                             label="chunglu_4m_g2.1_d16_mixed_16rhs"),
    "chunglu_4m_fp64": dict(cfg="c4_chunglu_4m", precision="fp64", k=16,
                            label="chunglu_4m_g2.1_d16_fp64_16rhs"),
}


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(family, workload):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{family}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(g, b, seconds_target=20.0):
    """The oracle as it stands, single thread, on whole steps of the same
    workload (setup + one solve), for about `seconds_target` seconds."""
    import oracle

    oracle.lib()
    steps = 0
    t0 = time.perf_counter()
    while True:
        h = oracle.Hierarchy(g, oracle.default_opts())
        x, st, it, rel, work = h.solve(b[:, 0], 1e-8, 500)
        del h
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds_target or el / steps * (steps + 1) > 2 * seconds_target:
            break
    return dict(value=steps / el, unit="solves/s", cores=1, kind="oracle",
                sample=f"{steps} full step(s) (setup + one solve to 1e-8) of the same "
                       f"workload, {el:.1f} s single-threaded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat_s18", choices=list(WORKLOADS))
    ap.add_argument("--latency-solves", type=int, default=100)
    ap.add_argument("--family", default="cheb", help="kernel family timed for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(a batch of right-hand sides or a pool of graphs would shard by replication; "
              "see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen as gg
    import paper_1705_06266_amd.lgmg as lg

    dev = torch.device("cuda:0")
    wl = WORKLOADS[args.workload]
    g = gg.config_graph(wl["cfg"])
    b_host = gg.config_rhs(wl["cfg"], g.n, wl["k"])
    rp = torch.as_tensor(g.row_ptr).to(dev)
    col = torch.as_tensor(g.col).to(dev)
    w = torch.as_tensor(g.w).to(dev)
    B = torch.as_tensor(b_host).to(dev)
    opts = lg.lg_default_opts(max_rhs=wl["k"],
                              precision=lg.LG_MIXED if wl["precision"] == "mixed" else lg.LG_FP64)
    torch.cuda.synchronize()

    def step():
        h = lg.lg_setup(rp, col, w, opts)
        X, info, st = lg.lg_solve(h, B, rtol=1e-8, max_iter=500)
        return h, info

    for _ in range(args.warmup):
        h, info = step()
        del h

    lg.lg_profile_enable(args.family)
    setup_ms, solve_ms, infos = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        h = lg.lg_setup(rp, col, w, opts)
        bm = time.perf_counter()
        X, info, st = lg.lg_solve(h, B, rtol=1e-8, max_iter=500)
        c = time.perf_counter()
        setup_ms.append((bm - a) * 1e3)
        solve_ms.append((c - bm) * 1e3)
        infos.append(info)
        assert st == 0 and all(i["rel_residual"] <= 1e-8 for i in info)
        del h
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, fam_ms, fam_bytes = lg.lg_profile_read()
    lg.lg_profile_enable(None)
    elapsed = t1 - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = args.steps * wl["k"] / elapsed

    # solve-only latency on a resident hierarchy
    h = lg.lg_setup(rp, col, w, opts)
    lat = []
    for _ in range(args.latency_solves):
        a = time.perf_counter()
        X, info, st = lg.lg_solve(h, B, rtol=1e-8, max_iter=500)
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)
    stats = lg.lg_hierarchy_stats(h)

    # fp64 SpMV bandwidth on the finest level (algorithmic bytes)
    n0, m0 = stats[0]["n"], stats[0]["nnz"]
    kk = 1 if wl["k"] == 1 else min(32, 1 << (wl["k"] - 1).bit_length())
    x = torch.randn(n0, kk, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(3):
        lg.lg_spmv(h, 0, x, y)
    lg.lg_profile_enable("spmm")
    reps = 50
    for _ in range(reps):
        lg.lg_spmv(h, 0, x, y)
    torch.cuda.synchronize()
    sp_n, sp_ms, sp_bytes = lg.lg_profile_read()
    lg.lg_profile_enable(None)
    spmv_gbs = sp_bytes / (sp_ms * 1e-3) / 1e9 if sp_ms > 0 else None

    achieved = fam_bytes / (fam_ms * 1e-3) / 1e9 if fam_ms > 0 else 0.0
    traffic = load_traffic(args.family, args.workload)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl["precision"] == "fp64" else "f32-cycle/f64-krylov",
        "data": "synthetic",
        "config": {"workload": wl["label"], "n": g.n, "nnz": g.nnz, "rhs": wl["k"], "rtol": 1e-8,
                   "step": "setup+solve", "levels": len(stats)},
        "roofline": {
            "bound": "hbm",
            "kernel_family": args.family,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "launches": launches,
            "avg_launch_ms": fam_ms / launches if launches else None,
            "algorithmic_bytes_per_launch": fam_bytes / launches if launches else None,
        },
        "setup_ms": float(np.median(setup_ms)),
        "solve_ms": float(np.median(solve_ms)),
        "iters": infos[-1][0]["iters"],
        "wda": infos[-1][0]["wda"],
        "solve_only": {"solves_per_s": wl["k"] * 1e3 / float(lat.mean()),
                       "p50_ms": float(np.percentile(lat, 50)),
                       "p99_ms": float(np.percentile(lat, 99)), "solves": int(lat.size)},
        "spmv_fp64_gbs": spmv_gbs,
        "spmv_fp64_ms": sp_ms / sp_n if sp_n else None,
        "spmv_fp64_rhs": kk,
    }
    del h
    if not args.no_cpu_baseline and args.workload in ("rmat_s18", "grid2d_64"):
        out["cpu_baseline"] = cpu_baseline(g, b_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
