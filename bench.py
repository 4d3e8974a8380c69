"""Benchmark of the triangle-counting hot path on one MI355X.

A step is one pass of the whole path over one graph already resident in HBM:
tc_build_csr (raw R-MAT pairs -> symmetric CSR) -> tc_orient (degree order)
-> tc_count_per_vertex (total and per-vertex counts).  The default workload is
R-MAT scale 24, edge factor 16 (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), seed 24,
with int64 row offsets; the scale-20 graph (seed 20, int32 offsets) is measured
after it and reported under "secondary".

Prints ONE JSON line.  `value` is GTEPS over the whole step: m (unique undirected
edges) / step time / 1e9.  Per-phase times come from HIP events recorded on the
stream the library launches on (torch's current stream).  The roofline object
covers the dominant kernel (the fused advance/filter/reduce count kernel).
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
DEFAULT_WORKLOAD = "rmat-s24-ef16"
SECONDARY_WORKLOAD = "rmat-s20-ef16"

WORKLOADS = {
    "rmat-s20-ef16": dict(kind="rmat", scale=20, ef=16, seed=20, offset_bytes=4),
    "rmat-s24-ef16": dict(kind="rmat", scale=24, ef=16, seed=24, offset_bytes=8),
    "er-n1024-m8192": dict(kind="er", n=1024, m=8192, seed=0, offset_bytes=4),
    # 4096 graphs, n log-uniform in [2^8, 2^16], average degree U(4, 64), ER/R-MAT alternating
    # int32 row offsets when the symmetric union fits them (it does: 2 * 8.07e8 < 2^31)
    "batch-4096": dict(kind="batch", count=4096, seed=4, offset_bytes=None),
    # Poisson request stream: batch-suite graphs plus 2% R-MAT scale 22 (edge factor 16)
    "serve-poisson": dict(kind="serve", pool=256, seed=5, large_scale=22, large_frac=0.02),
    # triangle listing (every triangle as a (u, v, w) row) on the scale-20 graph
    "list-rmat-s20-ef16": dict(kind="list", scale=20, ef=16, seed=20, offset_bytes=4),
    # the paper's own pipeline (NE filter + materialised two-iteration advance) against the
    # fused count, in id order and degree order, on the scale-20 graph
    "ablation-rmat-s20-ef16": dict(kind="ablation", scale=20, ef=16, seed=20, offset_bytes=4),
    # the 4-clique query on an R-MAT scale-18 graph (edge factor 16)
    "k4-rmat-s18-ef16": dict(kind="k4", scale=18, ef=16, seed=18, offset_bytes=4),
    # per-edge support (triangles on every edge) on the scale-20 graph
    "support-rmat-s20-ef16": dict(kind="support", scale=20, ef=16, seed=20, offset_bytes=4),
    # the segmented-intersection operator (merge path per DAG edge, count and support)
    # timed beside the wedge probe on the scale-20 graph
    "intersect-rmat-s20-ef16": dict(kind="intersect", scale=20, ef=16, seed=20, offset_bytes=4),
    # the diamond query (two triangles sharing an edge) on the scale-20 graph
    "diamond-rmat-s20-ef16": dict(kind="diamond", scale=20, ef=16, seed=20, offset_bytes=4),
    # labelled triangle queries, one of each shape ({a,a,a}, {a,a,b}, {a,b,c}), on the
    # scale-20 graph with four uniform vertex labels
    "labelled-rmat-s20-ef16": dict(kind="labelled", scale=20, ef=16, seed=20, offset_bytes=4,
                                   labels=4),
    # directed triangle queries (the 3-cycle and the transitive triangle) on the scale-20
    # R-MAT pairs read as arcs
    "directed-rmat-s20-ef16": dict(kind="directed", scale=20, ef=16, seed=20, offset_bytes=4),
    # triangle queries with edge labels (four uniform labels per pair) on the scale-20 graph
    "edge-labelled-rmat-s20-ef16": dict(kind="edge_labelled", scale=20, ef=16, seed=20,
                                        offset_bytes=4, labels=4),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-secondary", dest="secondary", action="store_false",
                    help=f"default workload only: skip the {SECONDARY_WORKLOAD} figures")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle check of the count")
    ap.add_argument("--batch-cache", metavar="PATH",
                    help="batch: load the generated graphs from PATH (.npz), or generate and save "
                         "them there (the generator's thousands of small launches make profiled "
                         "runs slow)")
    ap.add_argument("--count-only", action="store_true",
                    help="batch: only the packed count launch, K times (for profiling)")
    ap.add_argument("--cpu-budget-s", type=float, default=30.0)
    ap.add_argument("--requests", type=int, default=3000, help="serve: requests after warm-up")
    ap.add_argument("--qps", type=float, default=500.0, help="serve: Poisson arrival rate")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="serve: measure the mix's capacity (all requests queued at once), then "
                         "run 1000 warm-up + --requests requests at 0.3/0.5/0.7/0.9 of it; the "
                         "reported point is 0.7")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before timing, run a plain device copy of this many MiB (3 times) so a "
                         "counter profile can scale FETCH_SIZE/WRITE_SIZE by a known byte count")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="write the rocprofv3 --kernel-trace --stats CSV under DIR as a text summary "
                         "in profiles/ and exit (no GPU use)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the FETCH_SIZE / WRITE_SIZE counter runs under the two dirs as the "
                         "count kernel's traffic record in profiles/ and exit (no GPU use)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="write the rocprofv3 --pmc runs under the dirs (any counters) as a text "
                         "table of per-dispatch means for the library kernels in profiles/ and exit")
    ap.add_argument("--profile-command", action="append", default=[],
                    help="with --summarize-*: the command that produced the data (repeatable)")
    return ap.parse_args()


COUNT_SOURCES = ["paper_1909_02127_amd/csrc/count.hip", "paper_1909_02127_amd/csrc/tc_hash.h",
                 "paper_1909_02127_amd/csrc/tc_device.h"]


def count_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in COUNT_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(workload: str):
    """HBM bytes per count-kernel launch from the committed counter summary, or None when
    the summary is missing or was taken from different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"count_kernel_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_digest") != count_source_digest():
        return None
    return rec.get("traffic_bytes_per_launch")


def _profile_kernel(workload: str) -> str:
    """The dominant kernel a workload's profile summaries are named for."""
    kind = WORKLOADS[workload]["kind"]
    return {"k4": "k4_kernel", "intersect": "merge_kernel"}.get(kind, "count_kernel")


def _short_kernel_name(name: str) -> str:
    import re
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name)[:110]


def _csv_rows(directory: str, suffix: str):
    import csv
    import glob
    paths = glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)
    if not paths:
        raise SystemExit(f"no *{suffix} under {directory}")
    rows = []
    for p in paths:
        with open(p) as f:
            rows.extend(csv.DictReader(f))
    return rows


def summarize_trace(args) -> str:
    """profiles/<kernel>_<workload>_kernel_trace.txt from a --kernel-trace --stats run."""
    rows = _csv_rows(args.summarize_trace, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel-trace summary: workload {args.workload}, library kernels (tc::) only",
             "# command (repository root on the MI355X, after: cd /tmp && export TMPDIR=/tmp):"]
    lines += [f"#   {c}" for c in args.profile_command]
    lines.append("# calls  avg_us  min_us  max_us  total_ms  kernel")
    for r in rows:
        name = _short_kernel_name(r["Name"])
        if not name.startswith("tc::"):
            continue
        lines.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:11.2f} "
                     f"{float(r['MinNs']) / 1e3:11.2f} {float(r['MaxNs']) / 1e3:11.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.3f}  {name}")
    out = os.path.join(ROOT, "profiles",
                       f"{_profile_kernel(args.workload)}_{args.workload}_kernel_trace.txt")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return out


def summarize_counters(args) -> str:
    """profiles/count_kernel_<workload>_counters.txt: per-dispatch means of every collected
    counter for the library kernels, with the ratios read off them."""
    import collections
    vals = collections.defaultdict(list)
    for directory in args.summarize_counters:
        for r in _csv_rows(directory, "counter_collection.csv"):
            name = _short_kernel_name(r["Kernel_Name"])
            if name.startswith("tc::"):
                vals[(name, r["Counter_Name"])].append(float(r["Counter_Value"]))
    kernels = sorted({k for k, _ in vals})
    lines = [f"# rocprofv3 counters: workload {args.workload}, per-dispatch means, library kernels",
             "# commands (repository root on the MI355X, after: cd /tmp && export TMPDIR=/tmp):"]
    lines += [f"#   {c}" for c in args.profile_command]
    for k in kernels:
        cs = {c: sum(v) / len(v) for (kk, c), v in vals.items() if kk == k}
        lines.append(f"{k}  ({len(next(v for (kk, _), v in vals.items() if kk == k))} dispatches)")
        for c in sorted(cs):
            lines.append(f"    {c:28s} {cs[c]:20.1f}")
        if "SQ_LDS_BANK_CONFLICT" in cs and cs.get("SQ_INSTS_LDS"):
            lines.append(f"    {'bank-conflict cycles / LDS instr':28s} "
                         f"{cs['SQ_LDS_BANK_CONFLICT'] / cs['SQ_INSTS_LDS']:20.3f}")
        if "SQ_WAVE_CYCLES" in cs and cs.get("SQ_BUSY_CYCLES"):
            # SQ_WAVE_CYCLES sums the resident cycles of all waves in units of 4 cycles;
            # SQ_BUSY_CYCLES sums the busy cycles of the 32 shader engines: waves per SIMD
            # (1024 SIMDs) = 4 * WAVE_CYCLES / (BUSY_CYCLES / 32) / 1024
            lines.append(f"    {'waves per SIMD (mean)':28s} "
                         f"{cs['SQ_WAVE_CYCLES'] / cs['SQ_BUSY_CYCLES'] / 8:20.2f}")
        if "TCC_HIT_sum" in cs and "TCC_MISS_sum" in cs:
            tot = cs["TCC_HIT_sum"] + cs["TCC_MISS_sum"]
            if tot:
                lines.append(f"    {'L2 hit rate':28s} {cs['TCC_HIT_sum'] / tot:20.3f}")
    out = os.path.join(ROOT, "profiles",
                       f"{_profile_kernel(args.workload)}_{args.workload}_counters.txt")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return out


def calibration_copies(copies: list[float]) -> list[float]:
    """The counter values of the calibration copy: the benchmark copies the same buffer three
    times, so take the largest value that at least three copy dispatches share (within 2%);
    other copies of the run (a one-off clone of a larger array) are left out.  Falls back to
    the largest copies when no value repeats."""
    for v in sorted(copies, reverse=True):
        same = [c for c in copies if abs(c - v) <= 0.02 * v]
        if len(same) >= 3:
            return same
    top = max(copies)
    return [c for c in copies if c >= 0.95 * top]


def summarize_pmc(args) -> str:
    """profiles/count_kernel_<workload>_pmc.json: HBM bytes per count launch from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the counter reads for the calibration copy
    (a plain device copy of --calibrate-copy-mib MiB, the largest copy dispatches of the run)."""
    import collections
    rec = {"workload": args.workload, "source_digest": count_source_digest(),
           "commands": args.profile_command}
    per = {}
    for counter, directory in zip(("FETCH_SIZE", "WRITE_SIZE"), args.summarize_pmc):
        vals = collections.defaultdict(list)
        for r in _csv_rows(directory, "counter_collection.csv"):
            if r["Counter_Name"] == counter:
                vals[_short_kernel_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        copies = [v for k, vs in vals.items() if "copyBuffer" in k for v in vs]
        if not copies:
            raise SystemExit(f"{counter}: no calibration copy dispatches under {directory}")
        cal = calibration_copies(copies)
        cal_kib = sum(cal) / len(cal)
        per[counter] = (vals, cal_kib)
    mib = args.calibrate_copy_mib or 1024
    copy_bytes = mib << 20
    f_fac = copy_bytes / (per["FETCH_SIZE"][1] * 1024)
    w_fac = copy_bytes / (per["WRITE_SIZE"][1] * 1024)
    rec["calibration"] = {"copy_bytes": copy_bytes, "copy_fetch_kib": per["FETCH_SIZE"][1],
                          "copy_write_kib": per["WRITE_SIZE"][1], "fetch_factor": f_fac,
                          "write_factor": w_fac}
    # count_kernel<kind, wide, offset>: kind 1 = per-vertex, 0 = total only
    for key, kind in (("count_per_vertex", "1"), ("count_total_only", "0")):
        name = next((k for k in per["FETCH_SIZE"][0] if k.startswith(f"tc::count_kernel<{kind},")),
                    None)
        if name is None:
            continue
        fv, wv = per["FETCH_SIZE"][0][name], per["WRITE_SIZE"][0].get(name, [0.0])
        fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
        rec[key] = {"kernel": name, "dispatches": len(fv), "fetch_kib": fk, "write_kib": wk,
                    "fetch_bytes_scaled": fk * 1024 * f_fac, "write_bytes_scaled": wk * 1024 * w_fac,
                    "traffic_bytes_per_launch": fk * 1024 * f_fac + wk * 1024 * w_fac}
    # the per-vertex launch where the workload runs one (graphs), else the total-only one (batch)
    rec["traffic_bytes_per_launch"] = (rec.get("count_per_vertex") or
                                       rec.get("count_total_only") or {}).get(
                                           "traffic_bytes_per_launch")
    out = os.path.join(ROOT, "profiles", f"count_kernel_{args.workload}_pmc.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return out


def make_graph(spec, device):
    import graphgen
    if spec["kind"] == "rmat":
        return graphgen.rmat(spec["scale"], spec["ef"], spec["seed"], device=device)
    return graphgen.erdos_renyi(spec["n"], spec["m"], spec["seed"], device=device)


def algorithmic_bytes(dag_ptr, dag_col, n: int, offset_bytes: int, per_vertex: bool) -> dict:
    """Algorithmic bytes of one count launch (the roofline unit of the count kernel): what the
    wedge-probe method reads when no re-read is served by a cache -- 4 B per enumerated
    wedge id, 4 B + two row bounds per middle v of a surviving source, two row bounds per
    vertex for binning -- plus 8 B per per-vertex count written.  Caches serve part of the
    N+(v) re-reads, and whole cache lines are fetched for row bounds, so the measured
    traffic (FETCH_SIZE + WRITE_SIZE) can lie on either side of it."""
    import torch
    o = offset_bytes
    dp = (dag_ptr[1:] - dag_ptr[:-1]).to(torch.int64)
    src_ok = dp >= 2
    rows = torch.repeat_interleave(torch.arange(n, device=dag_ptr.device), dp)
    keep = src_ok[rows]
    mids = dag_col[: rows.numel()].to(torch.int64)[keep]
    wedges = int(dp[mids].sum().item())
    m_kept = int(keep.sum().item())
    b = 4 * wedges + (4 + 2 * o) * m_kept + 2 * o * n + 8 + (8 * n if per_vertex else 0)
    return {"bytes": b, "wedges": wedges, "middle_edges": m_kept}


def cpu_baseline(workload, s_host, d_host, n, m, frac: float | None = None):
    """The oracle (clean -> orient -> count with per-vertex) on the host cores.  The clean and
    orient take the whole graph; the count enumerates the sources whose ids lie below
    frac * n (ids are permuted by the generator, so that is a uniform sample of sources;
    frac = 1 for graphs of up to 2^22 vertices, 1/8 beyond) and its time is scaled by
    n / sources to the whole graph."""
    import numpy as np

    import oracle
    if frac is None:
        frac = 1.0 if n <= (1 << 22) else 1 / 8
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    rp, col = oracle.clean(n, s_host, d_host)
    t1 = time.perf_counter()
    dp, dc = oracle.orient(rp, col, oracle.ORDER_DEGREE)
    del col
    t2 = time.perf_counter()
    k = max(1, int(n * frac))
    total, _ = oracle.count(dp, dc, per_vertex=True, threads=threads, sources=k)
    t3 = time.perf_counter()
    t_count = (t3 - t2) * n / k
    whole = k >= n
    # the same count on one core, over a smaller prefix (an eighth of the sample)
    k1 = max(1, k // 8)
    t4 = time.perf_counter()
    oracle.count(dp, dc, per_vertex=True, threads=1, sources=k1)
    t_count1 = (time.perf_counter() - t4) * n / k1
    # restore the OpenMP thread count (an empty graph: nothing is counted)
    oracle.count(np.zeros(2, dtype=np.int64), np.zeros(0, dtype=np.int32), threads=threads)
    return {
        "value": m / (t1 - t0 + t2 - t1 + t_count) / 1e9,
        "unit": "GTEPS",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{workload}: clean {t1 - t0:.2f}s and orient {t2 - t1:.2f}s of the whole graph "
                   f"(one thread), count " + (f"{t3 - t2:.2f}s" if whole else
                   f"of the sources below {k} of {n} ({frac:.3g} of the ids, a uniform sample) "
                   f"{t3 - t2:.2f}s, scaled to {t_count:.2f}s for all") +
                   f" ({threads} OpenMP threads)"),
        "count_only_gteps": m / t_count / 1e9,
        "count_only_gteps_1core": m / t_count1 / 1e9,
        "count_1core_sample": f"the sources below {k1} of {n}, {time.perf_counter() - t4:.2f}s on one "
                              f"thread, scaled to {t_count1:.1f}s for all",
        "total": int(total) if whole else None,
    }


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def golden_for(workload: str):
    """The oracle's stored counts for a workload (tests/golden/make_*.py), or None."""
    spec = WORKLOADS[workload]
    if spec["kind"] != "rmat":
        return None
    path = os.path.join(ROOT, "tests", "golden",
                        f"rmat_s{spec['scale']}_ef{spec['ef']}_seed{spec['seed']}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def graph_line(args, workload, dev, *, cpu: bool) -> dict:
    """One graph: K timed steps of build -> orient -> count_per_vertex, the count kernel
    alone, its roofline, the oracle check and (cpu) the oracle baseline."""
    import hashlib

    import numpy as np
    import torch
    import paper_1909_02127_amd as tc

    spec = WORKLOADS[workload]
    s, d, n = make_graph(spec, dev)
    _say(f"{workload}: {s.numel()} raw pairs on {n} vertices")
    ob = spec["offset_bytes"]
    pipe = tc.Pipeline(n, s.numel(), offset_bytes=ob, order=tc.TC_ORDER_DEGREE, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        pipe.build(s, d)
        if ev:
            ev[1].record(stream)
        pipe.orient()
        if ev:
            ev[2].record(stream)
        pipe.count_per_vertex()
        if ev:
            ev[3].record(stream)

    if args.calibrate_copy_mib > 0:
        a = torch.empty(args.calibrate_copy_mib << 18, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    res = pipe.result(per_vertex=True)

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        step(evs[k])
    end.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = start.elapsed_time(end)
    ms_step = ms_total / args.steps
    phase = {"build_csr": [], "orient": [], "count_per_vertex": []}
    for e in evs:
        phase["build_csr"].append(e[0].elapsed_time(e[1]))
        phase["orient"].append(e[1].elapsed_time(e[2]))
        phase["count_per_vertex"].append(e[2].elapsed_time(e[3]))
    avg = {k: sum(v) / len(v) for k, v in phase.items()}
    _say(f"{workload}: {ms_step:.3f} ms per step {avg}")

    # The plain total-only count on the same DAG, timed the same way.
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pipe.count()
    torch.cuda.synchronize()
    c0.record(stream)
    for _ in range(args.steps):
        pipe.count()
    c1.record(stream)
    torch.cuda.synchronize()
    ms_count_total = c0.elapsed_time(c1) / args.steps
    total_only = pipe.result().total
    assert total_only == res.total, "tc_count and tc_count_per_vertex disagree"

    m, nnz = res.m, res.nnz
    alg = algorithmic_bytes(pipe.dag_ptr, pipe.dag_col, n, ob, per_vertex=True)
    t_cnt_s = avg["count_per_vertex"] / 1e3
    achieved = alg["bytes"] / t_cnt_s / 1e9
    traffic = counter_traffic(workload)

    out = {
        "metric": "GTEPS (bit-exact vs oracle)",
        "value": m / (ms_step / 1e3) / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "m": m, "nnz": nnz, "raw_pairs": s.numel(),
                   "offset_bytes": ob, "order": "degree", "per_vertex": True,
                   "seed": spec["seed"], "parallelism": "single-gpu"},
        "triangles": res.total,
        "triangles_per_s": res.total / (ms_step / 1e3),
        "phase_ms": avg,
        "count_only": {"ms_per_vertex": avg["count_per_vertex"], "ms_total_only": ms_count_total,
                       "gteps_per_vertex": m / t_cnt_s / 1e9,
                       "gteps_total_only": m / (ms_count_total / 1e3) / 1e9,
                       "triangles_per_s": res.total / t_cnt_s},
        "roofline": {"bound": "hbm", "kernel": "count_kernel (tc_count_per_vertex)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_gbps": traffic / t_cnt_s / 1e9 if traffic else None,
                     "algorithmic_bytes": alg["bytes"], "wedges": alg["wedges"]},
        "wall_s_timed": t_wall,
    }

    golden = golden_for(workload)
    if golden is not None:
        # the oracle's stored counts: the total and every t(v) through the array's digest
        t = np.ascontiguousarray(res.per_vertex.cpu().numpy().view(np.uint64), dtype="<u8")
        out["oracle_match"] = bool(
            res.total == golden["triangles"] and m == golden["m"]
            and hashlib.sha256(t.tobytes()).hexdigest() == golden["t_sha256"])
        out["oracle_check"] = "stored oracle counts (total and SHA-256 of every t(v))"
        del t
    if cpu or (golden is None and not args.no_check):
        hs, hd = s.cpu().numpy(), d.cpu().numpy()
        if cpu:
            cb = cpu_baseline(workload, hs, hd, n, m)
            total = cb.pop("total")
            if "oracle_match" not in out and total is not None:
                out["oracle_match"] = total == res.total
                out["oracle_check"] = "live oracle total"
            out["cpu_baseline"] = cb
        elif "oracle_match" not in out:
            import oracle
            out["oracle_match"] = oracle.triangles(n, hs, hd) == res.total
            out["oracle_check"] = "live oracle total"
    del pipe
    torch.cuda.empty_cache()
    return out


def oracle_prefix_baseline(fn, dp, dc, frac: float, value_of, unit: str, what: str) -> dict:
    """A single-threaded oracle function timed on the sources below frac * n.  Vertex
    ids are permuted by the generator, so the prefix is a uniform sample of sources."""
    n = dp.size - 1
    k = max(1, int(n * frac))
    t0 = time.perf_counter()
    r = fn(dp, dc, sources=k)
    dt = time.perf_counter() - t0
    return {"value": value_of(r, k) / dt, "unit": unit, "cores": 1, "kind": "oracle",
            "sample": f"sources below {k} of {n} ({frac:.3g} of the ids): {what} in {dt:.1f}s, "
                      f"one thread"}


def batch_main(args, spec):
    """Batched path vs the plain one-graph-per-launch path on the same packed graphs."""
    import numpy as np
    import torch

    import graphgen
    import oracle
    from paper_1909_02127_amd import tune as tuner
    from paper_1909_02127_amd.batch import BatchRunner, PackedBatch, PlainRunner

    def say(msg):
        print(msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    specs = graphgen.batch_suite_spec(spec["count"], seed=spec["seed"])
    graphs = None
    if args.batch_cache and os.path.exists(args.batch_cache):
        z = np.load(args.batch_cache)
        host = z["pairs"]
        # upload through a pinned staging buffer in chunks: DMA copies, no copy kernel
        pairs = torch.empty(host.shape, dtype=torch.int32, device="cuda")
        stage = torch.empty(1 << 26, dtype=torch.int32, pin_memory=True)
        for r in range(2):
            for a in range(0, host.shape[1], stage.numel()):
                k = min(stage.numel(), host.shape[1] - a)
                stage[:k].copy_(torch.from_numpy(host[r, a: a + k]))
                pairs[r, a: a + k].copy_(stage[:k])
        del host, stage
        off, ns = z["pair_off"].tolist(), z["n"].tolist()
        graphs = [(pairs[0, off[i]: off[i + 1]], pairs[1, off[i]: off[i + 1]], ns[i])
                  for i in range(len(ns))]
        say(f"loaded {len(graphs)} graphs from {args.batch_cache} ({time.perf_counter() - t0:.1f}s)")
    if graphs is None:
        graphs = []
        for i, g in enumerate(specs):
            graphs.append(graphgen.batch_graph(g, device="cuda"))
            if (i + 1) % 512 == 0:
                say(f"generated {i + 1}/{len(specs)} graphs ({time.perf_counter() - t0:.1f}s)")
        if args.batch_cache:
            off = np.cumsum([0] + [int(g[0].numel()) for g in graphs])
            np.savez(args.batch_cache, pair_off=off, n=np.array([g[2] for g in graphs]),
                     pairs=torch.stack([torch.cat([g[0] for g in graphs]),
                                        torch.cat([g[1] for g in graphs])]).cpu().numpy())
            say(f"saved to {args.batch_cache} ({time.perf_counter() - t0:.1f}s)")
    b = PackedBatch(graphs, offset_bytes=spec["offset_bytes"])
    say(f"packed: n={b.n} m={b.m} ({time.perf_counter() - t0:.1f}s)")
    if args.count_only:
        if args.calibrate_copy_mib > 0:  # a plain copy of known size, for the counter factor
            a = torch.empty(args.calibrate_copy_mib << 18, dtype=torch.int32, device="cuda")
            c = torch.empty_like(a)
            a.fill_(1)
            for _ in range(3):
                c.copy_(a)
            torch.cuda.synchronize()
            del a, c
        br = BatchRunner(b)
        br.enqueue()
        for _ in range(args.warmup):
            br.count_only()
        ms = _time_ms(br.count_only, args.steps, 0)
        totals, grand = br.results()
        print(json.dumps({"workload": args.workload, "ms_count": ms, "triangles": grand,
                          "offset_bytes": b.offset_bytes}), flush=True)
        return

    probe = BatchRunner(b)
    probe.enqueue()
    torch.cuda.synchronize()
    best, table = tuner.autotune(lambda t: BatchRunner.count_only(_with_tune(probe, t)),
                                 f"batch-4096-seed{spec['seed']}", use_cache=False)
    say(f"autotuned: {best}")
    del probe

    br = BatchRunner(b, tune=best)
    br.capture()
    for _ in range(args.warmup):
        br.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        br.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_batched = e0.elapsed_time(e1) / args.steps
    totals, grand = br.results()

    pr = PlainRunner(b)
    pr.enqueue()
    torch.cuda.synchronize()
    plain_steps = max(1, min(args.steps, 3))
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    p0.record()
    for _ in range(plain_steps):
        pr.enqueue()
    p1.record()
    torch.cuda.synchronize()
    ms_plain = p0.elapsed_time(p1) / plain_steps
    wall_plain = (time.perf_counter() - w0) / plain_steps * 1e3
    plain_totals = pr.results()

    # the dominant kernel alone (the batched count launch), timed with HIP events
    # on the stream it runs on, against its algorithmic bytes over the union DAG
    for _ in range(2):
        br.count_only()
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(args.steps):
        br.count_only()
    c1.record()
    torch.cuda.synchronize()
    ms_count = c0.elapsed_time(c1) / args.steps
    alg = algorithmic_bytes(br.dag_ptr, br.dag_col, b.n, b.offset_bytes, per_vertex=False)
    achieved = alg["bytes"] / (ms_count / 1e3) / 1e9

    rng = np.random.default_rng(0)
    sample = sorted(rng.choice(len(graphs), size=min(16, len(graphs)), replace=False).tolist())
    oracle_ok = all(
        oracle.triangles(graphs[i][2], graphs[i][0].cpu().numpy(), graphs[i][1].cpu().numpy())
        == totals[i] for i in sample)
    # every graph's total against the oracle's stored counts (tests/golden/make_batch4096.py)
    gpath = os.path.join(ROOT, "tests", "golden", f"batch{spec['count']}_seed{spec['seed']}.json")
    stored_ok = None
    if os.path.exists(gpath):
        with open(gpath) as f:
            stored_ok = [g["triangles"] for g in json.load(f)["graphs"]] == totals
    G = b.G
    cb = None
    if not args.no_cpu_baseline:
        # the oracle's whole pipeline per graph, graphs in batch order, for a bounded time
        host = [(g[2], g[0].cpu().numpy(), g[1].cpu().numpy()) for g in graphs]
        threads = oracle.max_threads()
        budget = min(args.cpu_budget_s, 20.0)
        done = 0
        w1 = time.perf_counter()
        while done < len(host) and time.perf_counter() - w1 < budget:
            n_i, s_i, d_i = host[done]
            oracle.triangles(n_i, s_i, d_i, threads=threads)
            done += 1
        dt = time.perf_counter() - w1
        cb = {"value": done / dt, "unit": "graphs/s", "cores": threads, "kind": "oracle",
              "sample": f"the first {done} of the {G} graphs in batch order, clean + orient + count "
                        f"each ({dt:.1f}s; count on {threads} OpenMP threads)"}
    out = {
        "metric": "batched graphs/s (bit-exact vs oracle)",
        "value": G / (ms_batched / 1e3),
        "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_batched,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "graphs": G, "n": b.n, "m": b.m,
                   "offset_bytes": b.offset_bytes, "order": "degree",
                   "parallelism": "single-gpu", "tune": best},
        "plain": {"ms_per_batch": ms_plain, "host_wall_ms_per_batch": wall_plain,
                  "graphs_per_s": G / (ms_plain / 1e3)},
        "speedup_vs_plain": ms_plain / ms_batched,
        "batched_gteps": b.m / (ms_batched / 1e3) / 1e9,
        "triangles": grand,
        "plain_equals_batched": plain_totals == totals,
        "oracle_sample_graphs": len(sample), "oracle_match": oracle_ok,
        "oracle_stored_all_graphs_match": stored_ok,
        "roofline": {"bound": "hbm", "kernel": "count_kernel (tc_count_batched)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(args.workload),
                     "algorithmic_bytes": alg["bytes"], "wedges": alg["wedges"],
                     "ms_count": ms_count},
        "autotune_table": table,
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def serve_main(args, spec):
    """Continuous-batching engine on a resident lane pool vs a plain engine (one request per
    launch, serialized, on one lane) on the same Poisson request stream."""
    import numpy as np
    import torch

    import graphgen
    import oracle
    from paper_1909_02127_amd import _lib
    from paper_1909_02127_amd.serve import DeviceExecutor, Engine, Lane, Request, lane_bytes, \
        plan_lanes

    rng = np.random.default_rng(spec["seed"])
    specs = graphgen.batch_suite_spec(4096, seed=4)
    pick = rng.choice(len(specs), size=spec["pool"], replace=False)
    pool = []
    for i in pick:
        s_, d_, n_ = graphgen.batch_graph(specs[int(i)], device="cuda")
        pool.append((s_.cpu().pin_memory(), d_.cpu().pin_memory(), n_))
    large = []
    for k in range(2):
        s_, d_, n_ = graphgen.rmat(spec["large_scale"], 16, 220 + k, device="cuda")
        large.append((s_.cpu().pin_memory(), d_.cpu().pin_memory(), n_))
    torch.cuda.synchronize()
    _say(f"pool: {len(pool)} graphs + {len(large)} scale-{spec['large_scale']} graphs")

    def stream(count, seed, qps=None):
        """Requests with Poisson arrivals at `qps` (None: args.qps; 0: all at time 0)."""
        qps = args.qps if qps is None else qps
        r = np.random.default_rng(seed)
        t, out = 0.0, []
        for i in range(count):
            t += float(r.exponential(1.0 / qps)) if qps > 0 else 0.0
            g = large[int(r.integers(len(large)))] if r.random() < spec["large_frac"] \
                else pool[int(r.integers(len(pool)))]
            out.append(Request(i, g[2], g[0], g[1], arrival=t))
        return out

    budget = 64 << 30
    big_pairs = max(int(g[0].numel()) for g in large)
    big_n = max(g[2] for g in large)
    # four lanes, one stream each: HIP gives a process four hardware queues by default, and a
    # stream that shares a queue with a large lane waits behind its graph in order
    lanes = plan_lanes(_lib, budget, small_lanes=2, small_pairs=24_000_000,
                       small_vertices=6_000_000, small_graphs=256, large_lanes=2,
                       large_pairs=big_pairs, large_vertices=big_n)
    ex = DeviceExecutor(lanes)
    _say(f"lanes: {[(ln.index, ln.large, ln.max_pairs, ln.bytes) for ln in lanes]}")

    def engine():
        return Engine(ex)

    sweep = None
    qps = args.qps
    if args.serve_sweep:
        # capacity of the mix: every request queued at time 0, completions per second
        cap_n = 3000
        cst = engine().run(stream(cap_n, 50, qps=0))
        capacity = cst.summary(warmup=cap_n // 10)["graphs_per_s"]
        _say(f"capacity: {capacity:.1f} graphs/s")
        sweep = {"capacity_graphs_per_s": capacity, "points": []}
        warm = 1000
        for frac in (0.3, 0.5, 0.9):
            pst_ = engine().run(stream(warm + args.requests, 60 + int(frac * 10),
                                       qps=frac * capacity))
            pt = pst_.summary(warmup=warm)
            pt["load"] = frac
            pt["qps"] = frac * capacity
            sweep["points"].append(pt)
            _say(f"load {frac}: {pt}")
        qps = 0.7 * capacity
    else:
        warm = max(1, args.requests // 10)
    eng = engine()
    reqs = stream(warm + args.requests, 51, qps=qps)
    st = eng.run(reqs)
    summ = st.summary(warmup=warm)
    _say(f"continuous batching at {qps:.1f} requests/s: {summ}")
    if sweep is not None:
        summ_pt = dict(summ, load=0.7, qps=qps)
        sweep["points"].insert(2, summ_pt)
    # exactness: every distinct graph that was served, total and t(v), against the oracle
    served = {}
    for r in reqs:
        served.setdefault(id(r.src), r)
    ok, checked = True, 0
    for r in served.values():
        if r.total is None:
            ok = False
            continue
        T, t = oracle.triangles(r.n, r.src.numpy(), r.dst.numpy(), per_vertex=True,
                                threads=oracle.max_threads())
        ok &= r.total == T and bool(np.array_equal(r.per_vertex, t))
        checked += 1
    same = True  # every request of one graph got the same counts
    for r in reqs:
        ref = served[id(r.src)]
        same &= r.total == ref.total and bool(np.array_equal(r.per_vertex, ref.per_vertex))
    _say(f"oracle: {checked} distinct graphs checked, match={ok}; repeats identical={same}")
    plain_n = max(1, min(args.requests // 3, 2000))
    plane = Lane(0, True, big_pairs, big_n, 1, lane_bytes(_lib, big_pairs, big_n, 1))
    peng = Engine(DeviceExecutor([plane]))
    preqs = stream(warm + plain_n, 51, qps=qps)
    pst = peng.run(preqs)
    psumm = pst.summary(warmup=warm)
    _say(f"plain: {psumm}")
    plain_same = all(a.total == b.total for a, b in zip(reqs, preqs))
    out = {
        "metric": "serving graphs/s (bit-exact vs oracle)",
        "value": summ["graphs_per_s"],
        "unit": "graphs/s",
        "n_gpus": 1, "steps": args.requests, "warmup": warm,
        "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "qps": qps, "requests": args.requests,
                   "warmup_requests": warm,
                   "pool": len(pool), "large_scale": spec["large_scale"],
                   "large_frac": spec["large_frac"], "budget_bytes": budget,
                   "lanes": [{"large": ln.large, "max_pairs": ln.max_pairs,
                              "max_vertices": ln.max_vertices, "max_graphs": ln.max_graphs,
                              "bytes": ln.bytes} for ln in lanes],
                   "parallelism": "single-gpu"},
        "p50_ms": summ["p50_ms"], "p99_ms": summ["p99_ms"], "serving": summ,
        "plain": psumm, "plain_requests": plain_n, "sweep": sweep,
        "oracle_match": bool(ok), "oracle_graphs_checked": checked,
        "repeats_identical": bool(same), "plain_equals_batched": bool(plain_same),
    }
    print(json.dumps(out), flush=True)


def list_main(args, spec):
    """tc_list_triangles on the resident DAG of an R-MAT graph: rows/s and its roofline."""
    import torch
    import paper_1909_02127_amd as tc

    dev = torch.device("cuda:0")
    s, d, n = make_graph(dict(spec, kind="rmat"), dev)
    ob = spec["offset_bytes"]
    pipe = tc.Pipeline(n, s.numel(), offset_bytes=ob, device=dev)
    pipe.enqueue(s, d)
    res = pipe.result()
    T = res.total
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        pipe.list_triangles(T)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        pipe.list_triangles(T)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    rows = pipe.listing()
    ok = rows.shape[0] == T
    cb = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        rp, col = oracle.clean(n, s.cpu().numpy(), d.cpu().numpy())
        dp, dc = oracle.orient(rp, col)
        if not args.no_check:
            ok = ok and oracle.count(dp, dc) == T
        if not args.no_cpu_baseline:
            cb = oracle_prefix_baseline(oracle.list_triangles, dp, dc, 1 / 4,
                                        lambda r, k: r.shape[0], "triangles/s",
                                        "every triangle listed")
    alg = algorithmic_bytes(pipe.dag_ptr, pipe.dag_col, n, ob, per_vertex=False)
    # two enumeration passes, 12 B per row written, a count and an offset per vertex
    b = 2 * alg["bytes"] + 12 * T + 16 * n
    achieved = b / (ms / 1e3) / 1e9
    out = {
        "metric": "triangles listed/s (count vs oracle)",
        "value": T / (ms / 1e3),
        "unit": "triangles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": res.m, "triangles": T,
                   "offset_bytes": ob, "order": "degree", "parallelism": "single-gpu"},
        "oracle_match": bool(ok),
        "roofline": {"bound": "hbm", "kernel": "count_kernel (listing: both passes)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": b},
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def support_main(args, spec):
    """tc_edge_support on the resident DAG of an R-MAT graph: edges/s and its roofline."""
    import numpy as np
    import torch
    import paper_1909_02127_amd as tc

    dev = torch.device("cuda:0")
    s, d, n = make_graph(dict(spec, kind="rmat"), dev)
    ob = spec["offset_bytes"]
    pipe = tc.Pipeline(n, s.numel(), offset_bytes=ob, device=dev)
    pipe.enqueue(s, d)
    res = pipe.result()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        pipe.edge_support()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        pipe.edge_support()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    sup = pipe.supports()
    T = res.total
    ok = int(sup.to(torch.int64).sum().item()) == 3 * T
    cb = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        rp, col = oracle.clean(n, s.cpu().numpy(), d.cpu().numpy())
        dp, dc = oracle.orient(rp, col)
        if not args.no_check:
            _, want = oracle.edge_support(dp, dc)
            ok = ok and np.array_equal(sup.cpu().numpy().view(np.uint32), want)
        if not args.no_cpu_baseline:
            cb = oracle_prefix_baseline(oracle.edge_support, dp, dc, 1 / 2,
                                        lambda r, k: int(dp[k]) / 1e9, "GTEPS",
                                        "the support of every edge")
    alg = algorithmic_bytes(pipe.dag_ptr, pipe.dag_col, n, ob, per_vertex=False)
    # the count's bytes, a 4-byte read-modify-write per triangle on (v, w), and per edge
    # the zeroing store plus the aggregated (u, v) and (u, w) read-modify-writes
    b = alg["bytes"] + 8 * T + 20 * res.m
    achieved = b / (ms / 1e3) / 1e9
    out = {
        "metric": "GTEPS of per-edge support (bit-exact vs oracle)",
        "value": res.m / (ms / 1e3) / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": res.m, "triangles": T,
                   "offset_bytes": ob, "order": "degree", "parallelism": "single-gpu"},
        "oracle_match": bool(ok),
        "roofline": {"bound": "hbm", "kernel": "count_kernel (support kind)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": b},
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def _time_ms(fn, steps: int, warmup: int) -> float:
    """Average ms of fn() over `steps` launches (after `warmup`), HIP events on torch's
    current stream, the stream the library launches on."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def merge_bytes(dag_ptr, dag_col, n: int, offset_bytes: int) -> dict:
    """Algorithmic bytes of the merge kernel of tc_segmented_intersect: every merge step
    loads one 4-byte list element (S = the sum over the edges with d+(u) >= 2 and
    d+(v) >= 1 of d+(u) + d+(v)), and every such edge its source, its v, its two scan
    entries and the row bounds of u and v."""
    import torch
    o = offset_bytes
    dp = (dag_ptr[1:] - dag_ptr[:-1]).to(torch.int64)
    rows = torch.repeat_interleave(torch.arange(n, device=dag_ptr.device), dp)
    du = dp[rows]
    dv = dp[dag_col[: rows.numel()].to(torch.int64)]
    live = (du >= 2) & (dv >= 1)
    steps = int((du + dv)[live].sum().item())
    edges = int(live.sum().item())
    return {"bytes": 4 * steps + (4 + 4 + 16 + 4 * o) * edges, "merge_steps": steps,
            "live_edges": edges}


def intersect_main(args, spec):
    """tc_segmented_intersect (merge path per DAG edge) against the wedge probe on the same
    resident DAG: total-only and per-edge support, both checked against the oracle."""
    import numpy as np
    import torch
    import paper_1909_02127_amd as tc

    dev = torch.device("cuda:0")
    s, d, n = make_graph(dict(spec, kind="rmat"), dev)
    ob = spec["offset_bytes"]
    pipe = tc.Pipeline(n, s.numel(), offset_bytes=ob, device=dev)
    pipe.enqueue(s, d)
    res = pipe.result()
    T = res.total
    ms_merge = _time_ms(lambda: pipe.intersect(), args.steps, args.warmup)
    T_merge = pipe.intersect_total()
    ms_merge_sup = _time_ms(lambda: pipe.intersect(support=True), args.steps, args.warmup)
    sup_merge = pipe.supports().clone()
    ms_hash = _time_ms(lambda: pipe.count(), args.steps, args.warmup)
    ms_hash_sup = _time_ms(lambda: pipe.edge_support(), args.steps, args.warmup)
    sup_hash = pipe.supports()
    ok = T_merge == T and torch.equal(sup_merge, sup_hash)
    cb = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        rp, col = oracle.clean(n, s.cpu().numpy(), d.cpu().numpy())
        dp, dc = oracle.orient(rp, col)
        if not args.no_check:
            T0, want = oracle.edge_support(dp, dc)
            ok = ok and T0 == T and np.array_equal(sup_merge.cpu().numpy().view(np.uint32), want)
        if not args.no_cpu_baseline:
            cb = oracle_prefix_baseline(
                lambda a, b, sources: oracle.count(a, b, threads=1, sources=sources), dp, dc, 1 / 2,
                                        lambda r, k: int(dp[k]) / 1e9, "GTEPS",
                                        "the count (node iterator, sorted merge per edge)")
    mb = merge_bytes(pipe.dag_ptr, pipe.dag_col, n, ob)
    # the kernel alone: the full call minus its edge-work pass and scan, timed separately
    # would need a split entry point; the whole call is reported and the roofline uses it
    achieved = mb["bytes"] / (ms_merge / 1e3) / 1e9
    out = {
        "metric": "GTEPS of the segmented intersection (bit-exact vs oracle)",
        "value": res.m / (ms_merge / 1e3) / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_merge,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": res.m, "triangles": T,
                   "offset_bytes": ob, "order": "degree", "parallelism": "single-gpu"},
        "ms": {"merge_total": ms_merge, "merge_support": ms_merge_sup,
               "hash_total": ms_hash, "hash_support": ms_hash_sup},
        "merge_over_hash": {"total": ms_merge / ms_hash, "support": ms_merge_sup / ms_hash_sup},
        "oracle_match": bool(ok),
        "roofline": {"bound": "hbm", "kernel": "tc_segmented_intersect (whole call)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes": mb["bytes"], "merge_steps": mb["merge_steps"]},
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def diamond_main(args, spec):
    """tc_count_diamonds on the resident DAG: diamonds/s, checked against the oracle."""
    import numpy as np
    import torch
    import paper_1909_02127_amd as tc

    dev = torch.device("cuda:0")
    s, d, n = make_graph(dict(spec, kind="rmat"), dev)
    ob = spec["offset_bytes"]
    pipe = tc.Pipeline(n, s.numel(), offset_bytes=ob, device=dev)
    pipe.enqueue(s, d)
    res = pipe.result()
    ms = _time_ms(lambda: pipe.diamonds(), args.steps, args.warmup)
    D = pipe.diamond_count()
    ok = None
    cb = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        hs, hd = s.cpu().numpy(), d.cpu().numpy()
        rp, col = oracle.clean(n, hs, hd)
        if not args.no_check:
            dp, dc = oracle.orient(rp, col)
            _, sup = oracle.edge_support(dp, dc)
            w = sup.astype(np.uint64)
            ok = D == int((w * (w - 1) // 2).sum())
        if not args.no_cpu_baseline:
            # the oracle's diamond enumeration on the edges whose lower end lies in a prefix
            # of the (permuted) ids, scaled to all of them
            k = n // 8
            t0 = time.perf_counter()
            oracle.count_diamonds(rp, col, sources=k)
            dt = (time.perf_counter() - t0) * n / k
            cb = {"value": res.m / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
                  "sample": f"the diamond enumeration for the edges whose lower end is below "
                            f"{k} of {n} ids, {dt * k / n:.1f}s, scaled to {dt:.1f}s for all"}
    # support enumeration (the count's bytes + support updates) and the C(s, 2) reduce
    alg = algorithmic_bytes(pipe.dag_ptr, pipe.dag_col, n, ob, per_vertex=False)
    b = alg["bytes"] + 8 * res.total + 20 * res.m + 4 * res.m
    achieved = b / (ms / 1e3) / 1e9
    out = {
        "metric": "diamonds/s (bit-exact vs oracle)",
        "value": D / (ms / 1e3),
        "unit": "diamonds/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": res.m, "diamonds": D,
                   "offset_bytes": ob, "order": "degree", "parallelism": "single-gpu"},
        "gteps": res.m / (ms / 1e3) / 1e9,
        "oracle_match": ok,
        "roofline": {"bound": "hbm", "kernel": "count_kernel (support kind) + C(s,2) reduce",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": b},
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


LABELLED_QUERIES = ((0, 0, 0), (1, 1, 2), (0, 1, 3))


def label_filter(dag_ptr, dag_col, n: int, labels, query):
    """The DAG edges whose label pair is a sub-multiset of the query (the filter of
    tc_count_labelled), as a CSR, and the filter's own algorithmic bytes: the labels of every
    source, the row bounds, out-lists and neighbour labels of the sources whose label is in
    the query, and the filtered DAG written."""
    import torch
    o = dag_ptr.element_size()
    a, b, c = sorted(query)
    dp = (dag_ptr[1:] - dag_ptr[:-1]).to(torch.int64)
    rows = torch.repeat_interleave(torch.arange(n, device=dag_ptr.device), dp)
    lu = labels[rows]
    lv = labels[dag_col[: rows.numel()].to(torch.int64)]
    lo, hi = torch.minimum(lu, lv), torch.maximum(lu, lv)
    fits = ((lo == a) & ((hi == b) | (hi == c))) | ((lo == b) & (hi == c))
    cand = (labels == a) | (labels == b) | (labels == c)
    e_cand = int(dp[cand].sum().item())
    kept_rows = rows[fits]
    cnt = torch.bincount(kept_rows, minlength=n)
    fptr = torch.zeros(n + 1, dtype=dag_ptr.dtype, device=dag_ptr.device)
    fptr[1:] = torch.cumsum(cnt, 0).to(dag_ptr.dtype)
    fcol = dag_col[: rows.numel()][fits].contiguous()
    m_kept = int(fcol.numel())
    b_filter = 4 * n + 2 * o * int(cand.sum().item()) + 8 * e_cand + o * (n + 1) + 4 * m_kept
    return fptr, fcol, m_kept, b_filter


def labelled_main(args, spec):
    """tc_count_labelled on the resident DAG with seeded vertex labels: one query of each
    shape per step, each count checked against the oracle."""
    import torch
    import graphgen
    import paper_1909_02127_amd as tc

    dev = torch.device("cuda:0")
    s, d, n = make_graph(dict(spec, kind="rmat"), dev)
    ob = spec["offset_bytes"]
    lab = graphgen.vertex_labels(n, spec["labels"], spec["seed"], device=dev)
    pipe = tc.Pipeline(n, s.numel(), offset_bytes=ob, device=dev)
    pipe.enqueue(s, d)
    res = pipe.result()
    per_q, counts, kept = {}, {}, {}
    for q in LABELLED_QUERIES:
        per_q[q] = _time_ms(lambda q=q: pipe.labelled(lab, q), args.steps, args.warmup)
        pipe.labelled(lab, q)
        counts[q] = pipe.labelled_count()
        kept[q] = int(pipe.labelled_kept.item())
    ms = sum(per_q.values())
    # algorithmic bytes: each filter pass plus the count of the DAG it writes
    b = 0
    for q in LABELLED_QUERIES:
        passes = [q]
        x = sorted(q)
        if (x[0] == x[1]) != (x[1] == x[2]):
            t = x[0] if x[0] == x[1] else x[2]
            passes.append((t, t, t))
        for pq in passes:
            fptr, fcol, _, bf = label_filter(pipe.dag_ptr, pipe.dag_col, n, lab, pq)
            b += bf + algorithmic_bytes(fptr, fcol, n, ob, per_vertex=False)["bytes"]
            del fptr, fcol
    achieved = b / (ms / 1e3) / 1e9
    ok = None
    cb = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        hs, hd, hl = s.cpu().numpy(), d.cpu().numpy(), lab.cpu().numpy()
        rp, col = oracle.clean(n, hs, hd)
        dp, dc = oracle.orient(rp, col)
        del rp, col
        t0 = time.perf_counter()
        want = {q: oracle.count_labelled(dp, dc, hl, q) for q in LABELLED_QUERIES}
        dt = time.perf_counter() - t0
        ok = want == counts
        if not args.no_cpu_baseline:
            cb = {"value": len(LABELLED_QUERIES) * res.m / dt / 1e9, "unit": "GTEPS", "cores": 1,
                  "kind": "oracle",
                  "sample": f"the oracle's labelled count of the {len(LABELLED_QUERIES)} queries "
                            f"on the whole oriented graph, {dt:.1f}s"}
    out = {
        "metric": "labelled triangle queries: GTEPS (m per query time, bit-exact vs oracle)",
        "value": len(LABELLED_QUERIES) * res.m / (ms / 1e3) / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": res.m, "labels": spec["labels"],
                   "offset_bytes": ob, "order": "degree", "parallelism": "single-gpu"},
        "queries": [{"query": list(q), "ms": per_q[q], "matches": counts[q],
                     "kept_edges": kept[q]} for q in LABELLED_QUERIES],
        "triangles": res.total,
        "oracle_match": ok,
        "roofline": {"bound": "hbm", "kernel": "label filter + count_kernel on the filtered DAG",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": b},
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


DIRECTED_QUERIES = {"cycle": (1, 2, 1), "transitive": (1, 1, 1)}


def directed_main(args, spec):
    """tc_count_directed on the resident DAG and arc directions: the 3-cycle and the
    transitive triangle per step.  Checked by the seven induced classes summing to the
    triangle count (the oracle takes minutes per query at this size; the GPU tests compare
    it with the GPU at smaller scales)."""
    import itertools
    import torch
    import paper_1909_02127_amd as tc

    dev = torch.device("cuda:0")
    s, d, n = make_graph(dict(spec, kind="rmat"), dev)
    ob = spec["offset_bytes"]
    pipe = tc.Pipeline(n, s.numel(), offset_bytes=ob, device=dev)
    pipe.enqueue(s, d)
    res = pipe.result()
    ms_dir = _time_ms(lambda: pipe.edge_directions(s, d), args.steps, args.warmup)
    per_q, counts = {}, {}
    for name, q in DIRECTED_QUERIES.items():
        per_q[name] = _time_ms(lambda q=q: pipe.directed(q), args.steps, args.warmup)
        pipe.directed(q)
        counts[name] = pipe.directed_count()
    ms = sum(per_q.values())
    ok = None
    if not args.no_check:
        classes = {}
        for codes in itertools.product((1, 2, 3), repeat=3):
            arcs = {(i, j) for (i, j), c in zip(((0, 1), (0, 2), (1, 2)), codes) if c & 1}
            arcs |= {(j, i) for (i, j), c in zip(((0, 1), (0, 2), (1, 2)), codes) if c & 2}
            key = min(tuple(sorted((p[i], p[j]) for i, j in arcs))
                      for p in itertools.permutations(range(3)))
            classes.setdefault(key, codes)
        tot = 0
        for q in classes.values():
            pipe.directed(q, induced=True)
            tot += pipe.directed_count()
        ok = tot == res.total
    cb = None
    if not args.no_cpu_baseline:
        import oracle
        hs, hd = s.cpu().numpy(), d.cpu().numpy()
        rp, col = oracle.clean(n, hs, hd)
        dp, dc = oracle.orient(rp, col)
        del rp, col
        k = n // 64
        t0 = time.perf_counter()
        want = oracle.count_directed(dp, dc, hs, hd, DIRECTED_QUERIES["cycle"], sources=k)
        dt = (time.perf_counter() - t0) * n / k
        cb = {"value": res.m / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
              "sample": f"the oracle's 3-cycle query over the triangles whose source id is "
                        f"below {k} of {n} ({want} matches), {dt * k / n:.1f}s, scaled to "
                        f"{dt:.1f}s for all"}
    # the count's bytes, plus the direction bytes: each edge's once as a middle (u, v) and
    # once beside its key in the source's table, and (v, w) once per closed wedge
    alg = algorithmic_bytes(pipe.dag_ptr, pipe.dag_col, n, ob, per_vertex=False)
    b = len(DIRECTED_QUERIES) * (alg["bytes"] + 2 * res.m + res.total)
    achieved = b / (ms / 1e3) / 1e9
    out = {
        "metric": "directed triangle queries: GTEPS (m per query time)",
        "value": len(DIRECTED_QUERIES) * res.m / (ms / 1e3) / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": res.m, "offset_bytes": ob,
                   "order": "degree", "parallelism": "single-gpu"},
        "queries": [{"query": name, "codes": list(DIRECTED_QUERIES[name]), "ms": per_q[name],
                     "matches": counts[name]} for name in DIRECTED_QUERIES],
        "edge_directions_ms": ms_dir,
        "triangles": res.total,
        "check": ok,
        "roofline": {"bound": "hbm", "kernel": "count_kernel (directed kind)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": b},
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


EDGE_LABELLED_QUERIES = ((0, 0, 0), (1, 1, 2), (0, 1, 3))


def edge_labelled_main(args, spec):
    """tc_count_edge_labelled on the resident DAG and edge labels: one query of each shape
    per step.  Checked by the counts of all label multisets summing to the triangle count
    (the oracle takes minutes per query at this size; the GPU tests compare it with the GPU
    at smaller scales)."""
    import itertools
    import numpy as np
    import torch
    import paper_1909_02127_amd as tc

    dev = torch.device("cuda:0")
    s, d, n = make_graph(dict(spec, kind="rmat"), dev)
    ob = spec["offset_bytes"]
    k = spec["labels"]
    lab = torch.as_tensor(np.random.default_rng(spec["seed"]).integers(0, k, size=s.numel()),
                          dtype=torch.uint8).to(dev)
    pipe = tc.Pipeline(n, s.numel(), offset_bytes=ob, device=dev)
    pipe.enqueue(s, d)
    res = pipe.result()
    ms_lab = _time_ms(lambda: pipe.edge_labels(s, d, lab), args.steps, args.warmup)
    per_q, counts = {}, {}
    for q in EDGE_LABELLED_QUERIES:
        per_q[q] = _time_ms(lambda q=q: pipe.edge_labelled(q), args.steps, args.warmup)
        pipe.edge_labelled(q)
        counts[q] = pipe.edge_labelled_count()
    ms = sum(per_q.values())
    ok = None
    if not args.no_check:
        tot = 0
        for q in itertools.combinations_with_replacement(range(k), 3):
            pipe.edge_labelled(q)
            tot += pipe.edge_labelled_count()
        ok = tot == res.total
    cb = None
    if not args.no_cpu_baseline:
        import oracle
        hs, hd, hl = s.cpu().numpy(), d.cpu().numpy(), lab.cpu().numpy()
        rp, col = oracle.clean(n, hs, hd)
        dp, dc = oracle.orient(rp, col)
        del rp, col
        ks = n // 64
        t0 = time.perf_counter()
        want = oracle.count_edge_labelled(dp, dc, hs, hd, hl, EDGE_LABELLED_QUERIES[2],
                                          sources=ks)
        dt = (time.perf_counter() - t0) * n / ks
        cb = {"value": res.m / dt / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
              "sample": f"the oracle's {list(EDGE_LABELLED_QUERIES[2])} query over the "
                        f"triangles whose source id is below {ks} of {n} ({want} matches), "
                        f"{dt * ks / n:.1f}s, scaled to {dt:.1f}s for all"}
    # per query: the filter (row bounds and every edge's label read, the kept columns read
    # and written with their labels, the new offsets written), then the count of the
    # filtered DAG with its label bytes (twice per kept edge, once per match)
    b = 0
    o = pipe.dag_ptr.element_size()
    dp = (pipe.dag_ptr[1:] - pipe.dag_ptr[:-1]).to(torch.int64)
    rows = torch.repeat_interleave(torch.arange(n, device=dev), dp)
    elab = pipe.edge_label[: rows.numel()]
    for q in EDGE_LABELLED_QUERIES:
        fits = torch.isin(elab, torch.tensor(sorted(set(q)), dtype=torch.uint8, device=dev))
        cnt = torch.bincount(rows[fits], minlength=n)
        fptr = torch.zeros(n + 1, dtype=pipe.dag_ptr.dtype, device=dev)
        fptr[1:] = torch.cumsum(cnt, 0).to(pipe.dag_ptr.dtype)
        fcol = pipe.dag_col[: rows.numel()][fits].contiguous()
        mk = int(fcol.numel())
        b += (2 * o * (n + 1) + res.m + 9 * mk
              + algorithmic_bytes(fptr, fcol, n, ob, per_vertex=False)["bytes"]
              + 2 * mk + counts[q])
        del fptr, fcol
    achieved = b / (ms / 1e3) / 1e9
    out = {
        "metric": "edge-labelled triangle queries: GTEPS (m per query time)",
        "value": len(EDGE_LABELLED_QUERIES) * res.m / (ms / 1e3) / 1e9,
        "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": res.m, "labels": k,
                   "offset_bytes": ob, "order": "degree", "parallelism": "single-gpu"},
        "queries": [{"query": list(q), "ms": per_q[q], "matches": counts[q]}
                    for q in EDGE_LABELLED_QUERIES],
        "edge_labels_ms": ms_lab,
        "triangles": res.total,
        "check": ok,
        "roofline": {"bound": "hbm", "kernel": "edge-label filter + count_kernel (coded kind)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": b},
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def ablation_main(args, spec):
    """Time the fused count and the paper's materialised two-iteration advance (with and
    without the NE filter) in both orders on one graph; all counts must agree."""
    import torch
    import paper_1909_02127_amd as tc
    from paper_1909_02127_amd import _lib

    dev = torch.device("cuda:0")
    s, d, n = make_graph(dict(spec, kind="rmat"), dev)
    ob = spec["offset_bytes"]
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    rows = []
    counts = set()
    reps = max(1, min(args.steps, 5))
    for order, name in ((tc.TC_ORDER_DEGREE, "degree"), (tc.TC_ORDER_ID, "id")):
        pipe = tc.Pipeline(n, s.numel(), offset_bytes=ob, order=order, device=dev)
        pipe.build(s, d)
        t_orient = timed(pipe.orient, reps)
        t_fused = timed(pipe.count, reps)
        res = pipe.result()
        counts.add(res.total)
        keep = torch.zeros(n, dtype=torch.uint8, device=dev)
        nstats = torch.zeros(3, dtype=torch.int64, device=dev)
        ws_ne = torch.empty(_lib.tc_ne_filter_workspace(n, 64), dtype=torch.uint8, device=dev)
        t_ne = timed(lambda: _lib.tc_ne_filter(n, pipe.row_ptr, pipe.col, keep, nstats, ws_ne), reps)
        cap = pipe.dag_col.numel()
        ws_b = torch.empty(_lib.tc_count_bfs_workspace(n, cap), dtype=torch.uint8, device=dev)
        bstats = torch.zeros(4, dtype=torch.int64, device=dev)
        for mask_name, mask in (("none", None), ("ne", keep)):
            t_bfs = timed(lambda: _lib.tc_count_bfs(n, pipe.dag_ptr, pipe.dag_col, bstats, ws_b,
                                                    frontier_capacity=cap, keep=mask), reps)
            st = bstats.cpu().tolist()
            counts.add(st[2])
            rows.append({"order": name, "ne_filter": mask_name, "ms_orient": t_orient,
                         "ms_fused_count": t_fused, "ms_ne_filter": t_ne if mask is not None else 0.0,
                         "ms_bfs_count": t_bfs, "frontier": st[0], "candidate_wedges": st[1],
                         "matches": st[2], "status": st[3],
                         "ne_kept": int(nstats[0].item()), "ne_rounds": int(nstats[1].item())})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        del pipe
    best_bfs = min(r["ms_bfs_count"] for r in rows)
    fused = min(r["ms_fused_count"] for r in rows if r["order"] == "degree")
    out = {
        "metric": "fused count speed-up over the materialised two-iteration advance",
        "value": best_bfs / fused, "unit": "x",
        "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": fused,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "offset_bytes": ob,
                   "parallelism": "single-gpu"},
        "counts_agree": len(counts) == 1, "triangles": counts.pop() if len(counts) == 1 else None,
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


def k4_main(args, spec):
    """tc_count_k4 on the resident DAG of an R-MAT graph: 4-cliques/s and edges/s."""
    import torch
    import paper_1909_02127_amd as tc
    from paper_1909_02127_amd import _lib

    dev = torch.device("cuda:0")
    s, d, n = make_graph(dict(spec, kind="rmat"), dev)
    pipe = tc.Pipeline(n, s.numel(), offset_bytes=spec["offset_bytes"], device=dev)
    pipe.enqueue(s, d)
    res = pipe.result()
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(_lib.tc_count_k4_workspace(n), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        _lib.tc_count_k4(n, pipe.dag_ptr, pipe.dag_col, total, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        _lib.tc_count_k4(n, pipe.dag_ptr, pipe.dag_col, total, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    k4 = int(total.item())
    # Algorithmic bytes of one launch: each source with d+ >= 3 reads its row bounds
    # and N+(u); each of its middles v its row bounds, and N+(v) when d+(v) >= 2;
    # each kept w (a triangle u -> v -> w with d+(v) >= 2) its row bounds and N+(w).
    o = spec["offset_bytes"]
    dplus = (pipe.dag_ptr[1:] - pipe.dag_ptr[:-1]).to(torch.int64)
    src3 = dplus >= 3
    rows_u = torch.repeat_interleave(torch.arange(n, device=dev), dplus)
    mid_ok = src3[rows_u]
    mids = pipe.dag_col.to(torch.int64)[: rows_u.numel()][mid_ok]
    b = int((2 * o + 4 * dplus[src3]).sum().item()) + 2 * o * int(mids.numel())
    b += 4 * int(dplus[mids][dplus[mids] >= 2].sum().item())
    del rows_u, mid_ok, mids
    pipe.list_triangles(res.total)
    tri = pipe.listing().to(torch.int64)
    keep = src3[tri[:, 0]] & (dplus[tri[:, 1]] >= 2)
    b += int((2 * o + 4 * dplus[tri[:, 2][keep]]).sum().item())
    del tri, keep
    achieved = b / (ms / 1e3) / 1e9
    ok = None
    cb = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        rp, col = oracle.clean(n, s.cpu().numpy(), d.cpu().numpy())
        dp, dc = oracle.orient(rp, col)
        if not args.no_check:
            ok = oracle.count_k4(dp, dc) == k4
        if not args.no_cpu_baseline:
            cb = oracle_prefix_baseline(oracle.count_k4, dp, dc, 1 / 2, lambda r, k: r,
                                        "4-cliques/s", "4-cliques counted")
    out = {
        "metric": "4-cliques/s (exact vs oracle)", "value": k4 / (ms / 1e3), "unit": "4-cliques/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": res.m, "triangles": res.total,
                   "k4": k4, "order": "degree", "parallelism": "single-gpu"},
        "gteps": res.m / (ms / 1e3) / 1e9, "oracle_match": ok,
        "roofline": {"bound": "hbm", "kernel": "k4_kernel", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes": b},
    }
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def _with_tune(runner, tune):
    runner.tune = tune
    return runner


def main():
    args = parse()
    if args.summarize_trace or args.summarize_pmc or args.summarize_counters:
        if args.summarize_trace:
            print(summarize_trace(args))
        if args.summarize_pmc:
            print(summarize_pmc(args))
        if args.summarize_counters:
            print(summarize_counters(args))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path "
              "runs on one GPU; sharding it over several is not implemented)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1909_02127_amd as tc

    spec = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if spec["kind"] == "batch":
        return batch_main(args, spec)
    if spec["kind"] == "serve":
        return serve_main(args, spec)
    if spec["kind"] == "list":
        return list_main(args, spec)
    if spec["kind"] == "support":
        return support_main(args, spec)
    if spec["kind"] == "ablation":
        return ablation_main(args, spec)
    if spec["kind"] == "k4":
        return k4_main(args, spec)
    if spec["kind"] == "intersect":
        return intersect_main(args, spec)
    if spec["kind"] == "diamond":
        return diamond_main(args, spec)
    if spec["kind"] == "labelled":
        return labelled_main(args, spec)
    if spec["kind"] == "directed":
        return directed_main(args, spec)
    if spec["kind"] == "edge_labelled":
        return edge_labelled_main(args, spec)
    out = graph_line(args, args.workload, dev, cpu=not args.no_cpu_baseline)
    if args.workload == DEFAULT_WORKLOAD and args.secondary:
        # the scale-20 graph as well: its own timed steps, roofline and oracle check
        sec = graph_line(args, SECONDARY_WORKLOAD, dev, cpu=False)
        out["secondary"] = {k: sec[k] for k in (
            "value", "unit", "ms_per_step", "config", "triangles", "triangles_per_s", "phase_ms",
            "count_only", "roofline", "oracle_match") if k in sec}
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
