"""Benchmark: solves/s of the whole hot path on one MI355X.

One step = one pass of the whole path over one batch of input already in HBM:
setup (validation, elimination, strength of connection, voting aggregation,
Galerkin products, Lanczos, coarsest pseudo-inverse) followed by the solve of
the batch's right-hand sides to a 1e-8 relative residual.  The default
workload is the largest single-GPU configuration: the 4M-vertex Chung-Lu
power-law graph (gamma 2.1, mean degree 16, largest degree 1e5, largest
component, U(0,1] weights) with 16 Gaussian right-hand sides, solved in FP64;
the mixed form (FP32 hierarchy values and cycle inside FP64 CG) is timed
beside it on the same inputs, both to the same final residual.

Prints one JSON line.  Besides the headline value it reports the solve-only
latency distribution on a resident hierarchy, the fp64 SpMV bandwidth of the
finest level, the kernel with the largest share of the step's GPU time against
the HBM roofline (HIP events around its launches inside the timed region), the
true residual recomputed on the host after the timed steps, and the CPU oracle
on a bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(ROOT, "profiles")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solves/s + p50/p99 latency to 1e-8 rel. residual; SpMV GB/s, mixed vs FP64"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1705_06266_amd/csrc/common.h", "paper_1705_06266_amd/csrc/ops.h",
                  "paper_1705_06266_amd/csrc/solve.hip", "paper_1705_06266_amd/csrc/setup.hip",
                  "paper_1705_06266_amd/csrc/prims.hip"]

# family: the profiler families whose launches are the roofline kernel (the
# kernel with the largest share of the step's GPU time in the workload's
# rocprofv3 summary); kernel: that kernel as rocprofv3 prints it, without the
# column-split kernels' unroll argument (its instances at every unroll count
# together, as the autotuner may pick another per level); companion: a second
# workload timed beside this one on the same inputs.
WORKLOADS = {
    "chunglu_4m": dict(cfg="chunglu_4m", precision="fp64", k=16,
                       label="chunglu_4m_g2.1_d16_fp64_16rhs", family="resid,resid64",
                       kernel="k_rows_col<lg::LapColOp<double, 16, 1, 0> >",
                       companion="chunglu_4m_mixed"),
    "chunglu_4m_mixed": dict(cfg="chunglu_4m", precision="mixed", k=16,
                             label="chunglu_4m_g2.1_d16_mixed_16rhs", family="spmv",
                             kernel="k_rows_col<lg::LapColOp<double, 16, 0, 2> >"),
    "rmat_s18": dict(cfg="rmat_s18", precision="fp64", k=1,
                     label="rmat_s18_ef16_lcc_u01_fp64_1rhs", family="resid,resid64",
                     kernel="k_rows<lg::LapOp<double, 1, 1, 0> >"),
    "grid2d_64": dict(cfg="grid2d_64", precision="fp64", k=1,
                      label="grid2d_64x64_unit_fp64_1rhs", family="spmv",
                      kernel="k_rows<lg::LapOp<double, 1, 0, 0> >"),
    "grid3d_128_mixed": dict(cfg="grid3d_128_loguniform", precision="mixed", k=32,
                             label="grid3d_128cube_loguniform_mixed_32rhs", family="spmv",
                             kernel="k_rows_col<lg::LapColOp<double, 32, 0, 2> >"),
    "grid3d_128_fp64": dict(cfg="grid3d_128_loguniform", precision="fp64", k=32,
                            label="grid3d_128cube_loguniform_fp64_32rhs", family="resid,resid64",
                            kernel="k_rows_col<lg::LapColOp<double, 32, 1, 0> >"),
}
DEFAULT_WORKLOAD = "chunglu_4m"


def _fam_tag(family):
    """File-name form of a family list."""
    return family.replace(",", "+")


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pmc_path(family, workload):
    return os.path.join(PROFILES, f"{_fam_tag(family)}_{workload}_pmc.txt")


def load_traffic(family, workload):
    """HBM bytes per launch of the roofline kernel from a committed rocprofv3
    counter summary (its "json:" line), if it was taken on the current kernel
    sources; else None."""
    path = pmc_path(family, workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        line = [ln for ln in f if ln.startswith("json: ")]
    if not line:
        return None
    rec = json.loads(line[-1][len("json: "):])
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def eigs_bench(lg, rp, col, w, opts, nev, reps=3):
    """Time of lg_eigs (nev smallest nonzero eigenpairs to tol 1e-8, block
    inverse subspace iteration) on a hierarchy of the same graph built with room
    for its block; setup is timed separately.  Median of reps calls."""
    import torch

    o = type(opts).from_buffer_copy(opts)
    block = 1
    while block < nev + 1:
        block *= 2
    o.max_rhs = max(o.max_rhs, block)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = lg.lg_setup(rp, col, w, o)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    ms, last = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = lg.lg_eigs(h, nev=nev, tol=1e-8, max_iter=200)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    lam, X, iters, resid, st = last
    del h
    return {"nev": nev, "block": block, "setup_ms": setup_ms, "eigs_ms": float(np.median(ms)),
            "block_iterations": int(iters), "lambda": [float(v) for v in lam],
            "max_rel_residual": float(np.max(np.asarray(resid) / np.maximum(np.abs(lam), 1e-300))),
            "status": int(st)}


def stream_roof(dev, elems=128 << 20, reps=8):
    """On-box HBM roofs next to the published 8 TB/s: device copy (read +
    write) and triad a = b + s c over 1 GiB fp64 arrays, best of reps, timed
    with events.  Measured after the timed steps (outside them)."""
    import torch

    a = torch.empty(elems, dtype=torch.float64, device=dev)
    b = torch.ones(elems, dtype=torch.float64, device=dev)
    c = torch.ones(elems, dtype=torch.float64, device=dev)
    nbytes = elems * 8
    res = {}
    for name, fn, moved in (("copy_gbs", lambda: a.copy_(b), 2 * nbytes),
                            ("triad_gbs", lambda: torch.add(b, c, alpha=3.0, out=a), 3 * nbytes)):
        fn()
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        res[name] = moved / (best * 1e-3) / 1e9
    del a, b, c
    torch.cuda.empty_cache()
    res["array_gib"] = elems * 8 / 2**30
    return res


def host_info():
    """CPU model (lscpu) and the cores this process may use."""
    model = None
    try:
        import subprocess

        for ln in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": avail, "os_cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(g, B, k, iters, max_sample_iters=30, single_thread_budget_s=25.0):
    """The oracle as it stands on the same workload: its OpenMP build (row
    loops on all of the threads OpenMP is given, bit-identical results) times
    one setup and one right-hand side solved to 1e-8; the oracle has no
    batching, so a step of k right-hand sides costs setup + k solves.  A solve
    that needs more than max_sample_iters iterations (the GPU's count, `iters`)
    is sampled: that many iterations are timed and scaled to the full count.
    The single-threaded build is timed the same way when the threaded run
    predicts it fits the budget."""
    import oracle

    cap = min(iters, max_sample_iters)

    def one(threaded):
        t0 = time.perf_counter()
        h = oracle.Hierarchy(g, oracle.default_opts(), threaded=threaded)
        setup_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        x, st, it, rel, work = h.solve(B[:, 0], 1e-8, cap if cap < iters else 500)
        sampled = st != 0 and cap < iters and it == cap  # stopped at the cap, not converged
        solve_s = (time.perf_counter() - t0) * (iters / it if sampled else 1.0)
        del h
        return {"threads": oracle.threads(threaded), "setup_s": setup_s, "solve_s_per_rhs": solve_s,
                "iters_timed": it, "iters_solve": iters if sampled else it,
                "rel_residual": rel, "status": st,
                "step_s": setup_s + k * solve_s, "solves_per_s": k / (setup_s + k * solve_s)}

    mt = one(True)
    print(f"oracle ({mt['threads']} threads): setup {mt['setup_s']:.1f} s, "
          f"solve {mt['solve_s_per_rhs']:.1f} s per right-hand side", file=sys.stderr, flush=True)
    st1 = None
    guess = (mt["setup_s"] + mt["solve_s_per_rhs"]) * min(mt["threads"], 4)
    if mt["threads"] == 1:
        st1 = mt
    elif guess <= single_thread_budget_s:
        st1 = one(False)
    solve_txt = (f"one of the {k} right-hand side(s) solved to 1e-8 ({mt['solve_s_per_rhs']:.1f} s, "
                 f"{mt['iters_solve']} iterations)" if mt["iters_timed"] == mt["iters_solve"] else
                 f"{mt['iters_timed']} CG iterations of one of the {k} right-hand side(s), scaled to "
                 f"the {mt['iters_solve']} iterations of a solve to 1e-8 "
                 f"({mt['solve_s_per_rhs']:.1f} s)")
    out = dict(value=mt["solves_per_s"], unit="solves/s", cores=mt["threads"], kind="oracle",
               sample=f"OpenMP oracle on {mt['threads']} threads: one setup ({mt['setup_s']:.1f} s) "
                      f"and {solve_txt}; value = {k} / (setup + {k} x solve)",
               setup_s=mt["setup_s"], solve_s_per_rhs=mt["solve_s_per_rhs"],
               iters=mt["iters_solve"], single_thread=st1, host=host_info())
    if st1 is None:
        out["single_thread"] = "not timed: predicted above the sample budget"
    return out


def host_true_residuals(g, B, X):
    """max over columns of ||b - L x|| / ||b|| (b projected to mean zero),
    recomputed on the host in fp64 from the input graph."""
    import scipy.sparse as sp

    A = sp.csr_matrix((g.w, g.col, g.row_ptr), shape=(g.n, g.n))
    d = np.asarray(A.sum(axis=1)).ravel()
    Bp = B - B.mean(axis=0)
    R = Bp - (d[:, None] * X - A @ X)
    return np.linalg.norm(R, axis=0) / np.linalg.norm(Bp, axis=0)


def energy_diff(g, Xa, Xb):
    """||xa - xb||_L / ||xb||_L per column (sqrt(x^T L x) from the edge list)."""
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    out = []
    for c in range(Xa.shape[1]):
        def en(x):
            dx = x[rows] - x[g.col]
            return np.sqrt(0.5 * np.dot(g.w, dx * dx))
        out.append(float(en(Xa[:, c] - Xb[:, c]) / en(Xb[:, c])))
    return out


# ------------------------------------------------------------ profile summaries
def _kernels_from_db(db_path):
    import sqlite3

    db = sqlite3.connect(db_path)
    return list(db.execute("select name, duration from kernels order by start"))


def _short(name):
    return name.split("(")[0].replace("void ", "").replace("lg::", "", 1).strip()


_UNROLL_ARG = re.compile(r"^(k_rows_col<.*>), \d+>$")


def _kernel_of(name):
    """A short kernel name without the column-split kernels' unroll argument:
    'k_rows_col<lg::LapColOp<double, 16, 1, 0>, 4>' -> 'k_rows_col<lg::LapColOp<double, 16, 1, 0> >'."""
    short = _short(name)
    m = _UNROLL_ARG.match(short)
    return m.group(1) + " >" if m else short


def pmc_summary(args):
    """Turns two rocprofv3 counter runs of this script (FETCH_SIZE, WRITE_SIZE,
    each with --calibration-copy) into HBM bytes per launch of the roofline
    kernel: every counter is scaled by what it reads for a copy of known size."""
    import sqlite3

    import csv

    wl = WORKLOADS[args.workload]
    out = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        base = os.path.join(args.pmc_summary, counter.lower())
        path = os.path.join(base, "run_counter_collection.csv")
        if os.path.exists(path):  # --output-format csv
            with open(path) as f:
                rows = [(r["Kernel_Name"], float(r["Counter_Value"])) for r in csv.DictReader(f)
                        if r["Counter_Name"] == counter]
        else:
            path = os.path.join(base, "run_results.db")
            db = sqlite3.connect(path)
            rows = list(db.execute(
                "select kernel_name, value from counters_collection where counter_name = ?",
                (counter,)))
        copy_kib = [v for n, v in rows if "copyBuffer" in n or "elementwise" in n]
        # the calibration copy moves 512 MiB each way: its largest dispatch
        cal = max(copy_kib)
        scale = (512 * 1024) / cal
        vals = [v for n, v in rows if _kernel_of(n) == wl["kernel"]]
        if not vals:
            raise SystemExit(f"{wl['kernel']} not found in {path}")
        out[counter] = dict(kib_per_launch_raw=float(np.mean(vals)), calibration_kib=cal,
                            scale=scale, launches=len(vals),
                            bytes_per_launch=float(np.mean(vals)) * scale * 1024)
    rec = dict(workload=args.workload, family=wl["family"], kernel=wl["kernel"],
               kernel_source_hash=kernel_source_hash(),
               read_bytes_per_launch=out["FETCH_SIZE"]["bytes_per_launch"],
               write_bytes_per_launch=out["WRITE_SIZE"]["bytes_per_launch"],
               hbm_bytes_per_launch=out["FETCH_SIZE"]["bytes_per_launch"]
               + out["WRITE_SIZE"]["bytes_per_launch"],
               counters=out, command=args.command)
    f_, w_ = out["FETCH_SIZE"], out["WRITE_SIZE"]
    lines = [f"# rocprofv3 byte counters, workload {wl['label']}", "",
             "commands (one run per counter):", "  " + args.command, "",
             f"kernel {wl['kernel']} ({f_['launches']} dispatches)",
             f"FETCH_SIZE {f_['kib_per_launch_raw']:.1f} KiB/dispatch; calibration copy of 512 MiB "
             f"reads {f_['calibration_kib']:.0f} KiB -> scale {f_['scale']:.4f} -> "
             f"{f_['bytes_per_launch'] / 1e6:.2f} MB read per dispatch",
             f"WRITE_SIZE {w_['kib_per_launch_raw']:.1f} KiB/dispatch; calibration copy of 512 MiB "
             f"writes {w_['calibration_kib']:.0f} KiB -> scale {w_['scale']:.4f} -> "
             f"{w_['bytes_per_launch'] / 1e6:.2f} MB written per dispatch",
             f"HBM traffic {rec['hbm_bytes_per_launch'] / 1e6:.2f} MB per dispatch",
             "", "json: " + json.dumps(rec)]
    os.makedirs(PROFILES, exist_ok=True)
    with open(pmc_path(wl["family"], args.workload), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_summary(args):
    """Writes a text summary of a rocprofv3 --kernel-trace --stats run of this
    script: per-kernel totals and averages, and the roofline kernel's row."""
    import csv

    wl = WORKLOADS[args.workload]
    stats = None
    for root, _, files in os.walk(args.trace_summary):
        for f in files:
            if f.endswith("kernel_stats.csv"):
                stats = os.path.join(root, f)
    if stats is None:
        raise SystemExit("no kernel_stats.csv under " + args.trace_summary)
    with open(stats) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics, workload {wl['label']}",
             "", "command:", "  " + args.command, "",
             f"{'total ms':>10} {'share':>6} {'calls':>7} {'avg us':>9}  kernel"]
    target = None
    for r in rows[:40]:
        name = _short(r["Name"])
        t = float(r["TotalDurationNs"])
        lines.append(f"{t / 1e6:10.3f} {100 * t / tot:5.1f}% {int(r['Calls']):7d} "
                     f"{float(r['AverageNs']) / 1e3:9.2f}  {name}")
    inst = [r for r in rows if _kernel_of(r["Name"]) == wl["kernel"]]
    lines.append("")
    if inst:
        calls = sum(int(r["Calls"]) for r in inst)
        total = sum(float(r["TotalDurationNs"]) for r in inst)
        lines.append(f"roofline kernel {wl['kernel']}: {calls} calls, "
                     f"average {total / calls / 1e3:.2f} us (rocprofv3)")
        if len(inst) > 1 or _short(inst[0]["Name"]) != wl["kernel"]:
            lines.append("  instances: " + "; ".join(
                f"{_short(r['Name'])} {int(r['Calls'])} calls, {float(r['AverageNs']) / 1e3:.2f} us"
                for r in inst))
    logs = [("same run under the profiler", args.bench_log),
            ("default run without the profiler", args.plain_log)]
    for what, log in logs:
        if not log:
            continue
        with open(log) as f:
            rec = json.loads([ln for ln in f if ln.startswith("{")][-1])
        # the workload's own line, or the companion object of the default run
        r = rec["roofline"] if rec["config"]["workload"] == wl["label"] else rec["mixed"]["roofline"]
        lines.append(f"{what}, HIP events in bench.py over the timed steps: {r['launches']} launches, "
                     f"average {r['avg_launch_ms'] * 1e3:.2f} us, "
                     f"{r['algorithmic_bytes_per_launch'] / 1e6:.2f} MB algorithmic per launch, "
                     f"{r['achieved']:.0f} GB/s")
    if args.bench_log and args.plain_log:
        lines.append("(kernel tracing adds time to the events that bracket each dispatch; the "
                     "kernel's own duration is the rocprofv3 figure, which the unprofiled events match)")
    os.makedirs(PROFILES, exist_ok=True)
    path = os.path.join(PROFILES, f"{_fam_tag(wl['family'])}_{args.workload}_kernel_stats.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def setup_summary(args):
    """Per-kernel breakdown of one setup from a rocprofv3 --kernel-trace run of
    this script: kernels from a setup's validation kernel up to the solve's
    first input kernel, the median setup of the run (by span)."""
    import csv

    wl = WORKLOADS[args.workload]
    trace = None
    for root, _, files in os.walk(args.setup_summary):
        for f in files:
            if f.endswith("kernel_trace.csv"):
                trace = os.path.join(root, f)
    if trace is None:
        raise SystemExit("no kernel_trace.csv under " + args.setup_summary)
    with open(trace) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    names = [_short(r["Kernel_Name"]) for r in rows]
    starts = [i for i, nm in enumerate(names) if nm == "k_validate"]
    setups = []
    for i0 in starts:
        ends = [i for i in range(i0, len(rows)) if names[i] == "k_pad_in"]
        if not ends:
            continue
        i1 = ends[0]
        span = (int(rows[i1 - 1]["End_Timestamp"]) - int(rows[i0]["Start_Timestamp"])) / 1e3
        setups.append((span, i0, i1))
    if not setups:
        raise SystemExit("no setup found in " + trace)
    setups.sort()
    span, i0, i1 = setups[len(setups) // 2]
    per, calls, busy = {}, {}, 0.0
    for i in range(i0, i1):
        d = (int(rows[i]["End_Timestamp"]) - int(rows[i]["Start_Timestamp"])) / 1e3
        busy += d
        per[names[i]] = per.get(names[i], 0.0) + d
        calls[names[i]] = calls.get(names[i], 0) + 1
    lines = [f"# rocprofv3 kernel breakdown of one setup, workload {wl['label']}", "",
             "command:", "  " + args.command, "",
             f"median of {len(setups)} setups in the trace: span {span:.1f} us from the first "
             f"kernel to the last, {i1 - i0} kernels, {busy:.1f} us of summed kernel time "
             "(the Lanczos steps run on a side stream, so kernels overlap; kernel tracing "
             "adds time between dispatches, so the span exceeds an unprofiled setup)", "",
             f"{'total us':>10} {'share':>6} {'calls':>6}  kernel"]
    for nm, t in sorted(per.items(), key=lambda x: -x[1])[:40]:
        lines.append(f"{t:10.1f} {100 * t / busy:5.1f}% {calls[nm]:6d}  {nm}")
    if args.plain_log:
        with open(args.plain_log) as f:
            rec = json.loads([ln for ln in f if ln.startswith("{")][-1])
        lines += ["", f"unprofiled run ({args.plain_log.split('/')[-1]}): setup median "
                      f"{rec['setup_ms']:.2f} ms per step"]
    os.makedirs(PROFILES, exist_ok=True)
    path = os.path.join(PROFILES, f"setup_{args.workload}_kernel_breakdown.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def serving_bench(args):
    """Serving workload: a seeded pool of 64 graphs (grids and R-MAT, 1e3-1e6
    vertices), requests of 1-8 right-hand sides on uniformly drawn graphs.
    Reports the mixed-precision continuous-batching server's saturated
    throughput and p50/p99 latency (submit to completion) under Poisson
    arrivals at fractions of that rate, next to plain FP64 single-column
    lg_solve calls on the same requests."""
    import threading

    import torch

    import graphgen as gg
    import paper_1705_06266_amd.lgmg as lg

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    pool = gg.serving_pool(count=args.pool)
    print(f"pool generated in {time.perf_counter() - t0:.1f} s: {len(pool)} graphs, "
          f"{sum(g.n for g in pool)} vertices", file=sys.stderr, flush=True)
    reqs = gg.serving_requests([g.n for g in pool], args.requests)
    rhs = [torch.as_tensor(gg.rhs(pool[gi].n, k, sd)).to(dev) for gi, k, sd in reqs]
    outs = [torch.empty_like(b) for b in rhs]
    torch.cuda.synchronize()

    srv = lg.Server(workers=args.workers, max_batch_rhs=32, precision=lg.LG_MIXED)
    gids = [srv.add_graph(g.row_ptr, g.col, g.w) for g in pool]
    # hierarchies: one request per graph builds and caches them all
    t0 = time.perf_counter()
    warm = [srv.submit(gids[i], torch.zeros(pool[i].n, 1, dtype=torch.float64, device=dev))
            for i in range(len(pool))]
    for r in warm:
        srv.wait(r)
    setup_s = time.perf_counter() - t0
    print(f"hierarchies built in {setup_s:.2f} s", file=sys.stderr, flush=True)

    def run(rate):
        """Submit every request (Poisson arrivals at `rate` requests/s, or all
        at once when rate is None); returns (seconds, latencies ms)."""
        rng = np.random.default_rng(11)
        gaps = rng.exponential(1.0 / rate, len(reqs)) if rate else np.zeros(len(reqs))
        ids = [None] * len(reqs)
        lat = [0.0] * len(reqs)

        def waiter():
            for i in range(len(reqs)):
                while ids[i] is None:
                    time.sleep(0.0002)
                lat[i] = srv.wait(ids[i])[3]

        th = threading.Thread(target=waiter)
        th.start()
        start = time.perf_counter()
        due = start
        for i, (gi, k, _) in enumerate(reqs):
            due += gaps[i]
            while time.perf_counter() < due:
                pass
            ids[i] = srv.submit(gids[gi], rhs[i], outs[i])
        th.join()
        return time.perf_counter() - start, np.array(lat)

    cols = sum(k for _, k, _ in reqs)
    sat_s, sat_lat = run(None)
    sat_req_rate = len(reqs) / sat_s
    st = srv.stats()
    sweep = []
    for frac in (0.25, 0.5, 0.75, 1.0, 1.25):
        el, lat = run(frac * sat_req_rate)
        sweep.append({"load": frac, "offered_req_per_s": frac * sat_req_rate,
                      "solves_per_s": cols / el, "p50_ms": float(np.percentile(lat, 50)),
                      "p99_ms": float(np.percentile(lat, 99))})
        print(f"load {frac}: {sweep[-1]}", file=sys.stderr, flush=True)
    srv.close()

    # plain FP64 single-column solves of the same requests, one at a time
    hs = {}
    base_n = min(len(reqs), args.baseline_requests)
    used = sorted({reqs[i][0] for i in range(base_n)})
    for gi in used:
        g = pool[gi]
        hs[gi] = lg.lg_setup(torch.as_tensor(g.row_ptr).to(dev), torch.as_tensor(g.col).to(dev),
                             torch.as_tensor(g.w).to(dev), lg.lg_default_opts(max_rhs=1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    base_cols = 0
    for i in range(base_n):
        gi, k, _ = reqs[i]
        for c in range(k):
            lg.lg_solve(hs[gi], rhs[i][:, c:c + 1].contiguous())
            base_cols += 1
    base_s = time.perf_counter() - t0
    out = {
        "metric": "serving: solves/s + p50/p99 latency to 1e-8 (continuous batching, mixed)",
        "value": cols / sat_s, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "data": "synthetic",
        "config": {"workload": f"serving_pool{args.pool}_grids_rmat_1e3-1e6_1-8rhs",
                   "requests": len(reqs), "rhs": cols, "workers": args.workers,
                   "max_batch_rhs": 32, "precision": "f32-cycle/f64-krylov"},
        "saturated": {"seconds": sat_s, "req_per_s": sat_req_rate,
                      "p50_ms": float(np.percentile(sat_lat, 50)),
                      "p99_ms": float(np.percentile(sat_lat, 99)),
                      "batches": st["batches"], "batched_columns": st["batched_columns"]},
        "poisson_sweep": sweep,
        "hierarchy_build_s": setup_s,
        "fp64_single_rhs_baseline": {"solves_per_s": base_cols / base_s, "rhs": base_cols},
        "speedup_vs_fp64_single_rhs": (cols / sat_s) / (base_cols / base_s),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=list(WORKLOADS) + ["serving"])
    ap.add_argument("--pool", type=int, default=64, help="serving: graphs in the pool")
    ap.add_argument("--requests", type=int, default=400, help="serving: requests per run")
    ap.add_argument("--workers", type=int, default=8, help="serving: server workers")
    ap.add_argument("--baseline-requests", type=int, default=120,
                    help="serving: requests replayed as FP64 single-column solves")
    ap.add_argument("--latency-solves", type=int, default=None,
                    help="solve-only latency samples (default 100, 20 above 2^24 nnz)")
    ap.add_argument("--no-companion", action="store_true",
                    help="skip the companion workload (the mixed form beside the FP64 default)")
    ap.add_argument("--family", default=None, help="kernel family timed for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cycle", type=int, default=None, choices=(1, 2),
                    help="1: V-cycle under CG (default), 2: K-cycle under flexible CG")
    ap.add_argument("--eigs", type=int, default=0, metavar="NEV",
                    help="also time lg_eigs for the NEV smallest nonzero eigenpairs (tol 1e-8) "
                         "on a hierarchy of the workload's graph")
    ap.add_argument("--no-hub-rows", dest="hub_rows", action="store_false",
                    help="skip the extra solve that times hub rows apart (counter and trace runs: "
                         "its split launches would mix into the roofline kernel's dispatches)")
    ap.add_argument("--no-stream-roof", action="store_true",
                    help="skip the on-box copy / triad bandwidth measurement")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="end with a 512 MiB device copy (scale for rocprofv3 byte counters)")
    ap.add_argument("--pmc-summary", default=None,
                    help="directory with fetch_size/ and write_size/ rocprofv3 runs: write the "
                         "traffic summary and exit (no GPU)")
    ap.add_argument("--trace-summary", default=None,
                    help="directory of a rocprofv3 --stats csv run: write the summary and exit")
    ap.add_argument("--setup-summary", default=None,
                    help="directory of a rocprofv3 --kernel-trace csv run: write the per-kernel "
                         "breakdown of one setup and exit")
    ap.add_argument("--graphs", type=int, default=None, choices=[0, 1],
                    help="replay the cycle as a captured HIP graph (default: the library's)")
    ap.add_argument("--autotune", type=int, default=None, choices=[0, 1],
                    help="time row-lane shifts per level at setup (default: the library's)")
    ap.add_argument("--merge-path", type=int, default=None, choices=[0, 1, 2],
                    help="one-column products: 0 class rows, 1 tuner's choice, 2 merge path")
    ap.add_argument("--command", default="", help="command line recorded in summaries")
    ap.add_argument("--bench-log", default=None, help="bench output of the profiled run (summaries)")
    ap.add_argument("--plain-log", default=None, help="bench output of a run without the profiler (summaries)")
    args = ap.parse_args()

    if args.pmc_summary:
        return pmc_summary(args)
    if args.trace_summary:
        return trace_summary(args)
    if args.setup_summary:
        return setup_summary(args)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(batches of right-hand sides or a pool of graphs would shard by keeping a "
              "replica of each hierarchy per GPU)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serving":
        return serving_bench(args)

    import torch

    import graphgen as gg
    import paper_1705_06266_amd.lgmg as lg

    dev = torch.device("cuda:0")
    wl = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    g = gg.config_graph(wl["cfg"])
    b_host = gg.config_rhs(wl["cfg"], g.n, wl["k"])
    say(f"graph {wl['cfg']}: n={g.n} nnz={g.nnz}, generated in {time.perf_counter() - t0:.1f} s")
    rp = torch.as_tensor(g.row_ptr).to(dev)
    col = torch.as_tensor(g.col).to(dev)
    w = torch.as_tensor(g.w).to(dev)
    B = torch.as_tensor(b_host).to(dev)
    latency_solves = args.latency_solves
    if latency_solves is None:
        latency_solves = 100 if g.nnz < (1 << 24) else 20

    out = measure(args, lg, dev, g, b_host, rp, col, w, B, args.workload, args.family,
                  latency_solves)
    comp = wl.get("companion")
    if comp and not args.no_companion:
        mo = measure(args, lg, dev, g, b_host, rp, col, w, B, comp, None, latency_solves)
        X64, Xmx = out.pop("_X"), mo.pop("_X")
        ed = energy_diff(g, Xmx[:, [0, -1]], X64[:, [0, -1]])
        out["mixed"] = {k: mo[k] for k in ("value", "ms_per_step", "dtype", "setup_ms", "solve_ms",
                                           "iters", "wda", "roofline", "solve_only",
                                           "host_true_rel_residual_max", "hierarchy_bytes")
                        if k in mo}
        out["mixed"]["workload"] = WORKLOADS[comp]["label"]
        out["mixed"]["energy_norm_diff_vs_fp64"] = max(ed)
        out["mixed_speedup_vs_fp64"] = mo["value"] / out["value"]
    else:
        out.pop("_X", None)
    if args.eigs:
        out["eigs"] = eigs_bench(lg, rp, col, w, out.pop("_opts"), args.eigs)
    out.pop("_opts", None)
    if not args.no_stream_roof and not args.calibration_copy:  # (counter runs calibrate on a copy)
        out["stream_roof"] = stream_roof(dev)
    if args.calibration_copy:
        src = torch.empty(64 << 20, dtype=torch.float64, device=dev)  # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        say("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(g, b_host, wl["k"], out["iters"])
    print(json.dumps(out), flush=True)


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def measure(args, lg, dev, g, b_host, rp, col, w, B, workload, family, latency_solves):
    """Warm-up and timed steps of one workload on resident inputs, then
    (outside the timed region) the host residual check, solve-only latency and
    the finest-level fp64 SpMV rate."""
    import torch

    wl = WORKLOADS[workload]
    family = family or wl["family"]
    opts = lg.lg_default_opts(max_rhs=wl["k"],
                              precision=lg.LG_MIXED if wl["precision"] == "mixed" else lg.LG_FP64)
    if args.graphs is not None:
        opts.graphs = args.graphs
    if args.autotune is not None:
        opts.autotune = args.autotune
    if args.merge_path is not None:
        opts.merge_path = args.merge_path
    if args.cycle is not None:
        opts.cycle = args.cycle
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        h = lg.lg_setup(rp, col, w, opts)
        X, info, st = lg.lg_solve(h, B, rtol=1e-8, max_iter=500)
        del h
    say(f"{workload}: {args.warmup} warm-up step(s) done; timing {args.steps}")

    lg.lg_profile_enable(family)
    setup_ms, solve_ms, infos = [], [], []
    X = None
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
    say(f"{workload}: {ms_per_step:.2f} ms per step, {value:.2f} solves/s")

    # the last timed step's solutions, checked on the host (outside the timed region)
    Xh = X.cpu().numpy()
    true_rel = host_true_residuals(g, b_host, Xh)
    assert np.all(true_rel <= 1e-8 * 1.001), true_rel.max()

    # solve-only latency on a resident hierarchy
    h = lg.lg_setup(rp, col, w, opts)
    lat = []
    for _ in range(latency_solves):
        a = time.perf_counter()
        X, info, st = lg.lg_solve(h, B, rtol=1e-8, max_iter=500)
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)
    stats = lg.lg_hierarchy_stats(h)
    hier_bytes = lg.lg_hierarchy_bytes(h)

    # hub and split rows (a workgroup or more per row), timed as launches of
    # their own in one more solve; every row is reduced as in the timed steps
    hub = None
    if args.hub_rows and any(s["n_hub"] for s in stats):
        lg.lg_profile_enable("hubs")
        torch.cuda.synchronize()
        a = time.perf_counter()
        lg.lg_solve(h, B, rtol=1e-8, max_iter=500)
        torch.cuda.synchronize()
        solve_ms_h = (time.perf_counter() - a) * 1e3
        hn, hms, _ = lg.lg_profile_read()
        lg.lg_profile_enable(None)
        hub = {"launches": hn, "ms_per_solve": hms, "solve_ms": solve_ms_h,
               "share_of_solve": hms / solve_ms_h if solve_ms_h > 0 else None,
               "rows_per_level": [s["n_hub"] for s in stats]}

    # fp64 SpMV bandwidth on the finest level (algorithmic bytes), lg_spmv's own kernels
    n0 = stats[0]["n"]
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
    del x, y
    # the same product on every level (hub rows are processed in the same launch
    # as the other rows), and the fraction each elimination level removes
    by_level = []
    for l, s in enumerate(stats):
        if s["type"] == lg.LG_LEVEL_COARSEST:
            continue
        xl = torch.randn(s["n"], kk, dtype=torch.float64, device=dev)
        yl = torch.empty_like(xl)
        for _ in range(3):
            lg.lg_spmv(h, l, xl, yl)
        lg.lg_profile_enable("spmm")
        for _ in range(20):
            lg.lg_spmv(h, l, xl, yl)
        torch.cuda.synchronize()
        ln, lms, lbytes = lg.lg_profile_read()
        lg.lg_profile_enable(None)
        row = {"level": l, "type": "elim" if s["type"] == lg.LG_LEVEL_ELIM else "agg",
               "n": s["n"], "nnz": s["nnz"], "hub_rows": s["n_hub"],
               "spmm_us": lms / ln * 1e3 if ln else None,
               "spmm_gbs": lbytes / (lms * 1e-3) / 1e9 if lms > 0 else None}
        if s["type"] == lg.LG_LEVEL_ELIM:
            row["eliminated_fraction"] = 1.0 - s["nc"] / s["n"]
        by_level.append(row)
        del xl, yl
    del h

    achieved = fam_bytes / (fam_ms * 1e-3) / 1e9 if fam_ms > 0 else 0.0
    traffic = load_traffic(family, workload) if family == wl["family"] else None
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
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": wl["kernel"] if family == wl["family"] else None,
            "kernel_family": family,
            "launches": launches,
            "avg_launch_ms": fam_ms / launches if launches else None,
            "algorithmic_bytes_per_launch": fam_bytes / launches if launches else None,
        },
        "setup_ms": float(np.median(setup_ms)),
        "solve_ms": float(np.median(solve_ms)),
        "iters": infos[-1][0]["iters"],
        "iters_per_rhs": [i["iters"] for i in infos[-1]],
        "wda": infos[-1][0]["wda"],
        "host_true_rel_residual_max": float(true_rel.max()),
        "spmv_fp64_gbs": spmv_gbs,
        "spmv_fp64_ms": sp_ms / sp_n if sp_n else None,
        "spmv_fp64_rhs": kk,
        "spmv_fp64_by_level": by_level,
        "hub_rows": hub,
        "hierarchy_bytes": hier_bytes,
        "levels": [(s["type"], s["n"], s["nnz"], s["lane_shift"], s["col_shift"], s["merge"],
                    s["col_unroll"]) for s in stats],
        "_X": Xh,
        "_opts": opts,
    }
    if lat.size:
        out["solve_only"] = {"solves_per_s": wl["k"] * 1e3 / float(lat.mean()),
                             "p50_ms": float(np.percentile(lat, 50)),
                             "p99_ms": float(np.percentile(lat, 99)), "solves": int(lat.size)}
    return out

if __name__ == "__main__":
    main()
