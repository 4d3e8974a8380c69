"""Host-side checks of bench.py (no GPU): the one-GPU guard, the rule that the counter-derived
HBM traffic is reported only for the kernel sources it was measured on, and the profile
summaries written from rocprofv3 CSV output (synthetic CSVs with the profiler's column names)."""
import argparse
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

COUNT1 = ("void tc::(anonymous namespace)::count_kernel<1, false, int>(int const*, int const*, "
          "int const*, tc::(anonymous namespace)::CountState*, unsigned long*, unsigned long*, "
          "tc::(anonymous namespace)::CountArgs)")
COUNT0 = COUNT1.replace("count_kernel<1,", "count_kernel<0,")
COPY = "__amd_rocclr_copyBuffer"
TORCH = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<long> >(int)"


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


@pytest.fixture
def fake_root(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_for_the_sources_it_was_measured_on(fake_root, monkeypatch):
    assert bench.counter_traffic("rmat-s20-ef16") is None  # no record
    rec = {"source_digest": "abc", "traffic_bytes_per_launch": 1.5e10}
    (fake_root / "profiles" / "count_kernel_rmat-s20-ef16_pmc.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "count_source_digest", lambda: "abc")
    assert bench.counter_traffic("rmat-s20-ef16") == 1.5e10
    monkeypatch.setattr(bench, "count_source_digest", lambda: "abd")
    assert bench.counter_traffic("rmat-s20-ef16") is None


def test_source_digest_covers_the_count_kernel_sources():
    d = bench.count_source_digest()
    assert len(d) == 16 and int(d, 16) >= 0
    names = {os.path.basename(p) for p in bench.COUNT_SOURCES}
    assert {"count.hip", "tc_hash.h", "tc_device.h"} <= names
    for rel in bench.COUNT_SOURCES:
        assert os.path.exists(os.path.join(ROOT, rel)), rel


def test_trace_summary_keeps_library_kernels_sorted_by_total(fake_root):
    header = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs",
              "StdDev"]
    rows = [[TORCH, 200, 9_000_000, 45_000.0, 8.0, 41_000, 53_000, 2_000.0],
            [COUNT0, 6, 15_000_000, 2_500_000.0, 30.0, 2_400_000, 2_600_000, 1.0],
            [COUNT1, 6, 16_800_000, 2_800_000.0, 32.0, 2_700_000, 2_960_000, 1.0]]
    _write_csv(str(fake_root / "kt" / "run_kernel_stats.csv"), header, rows)
    args = argparse.Namespace(summarize_trace=str(fake_root / "kt"), workload="rmat-s20-ef16",
                              profile_command=["rocprofv3 --kernel-trace --stats -- python3 bench.py"])
    out = bench.summarize_trace(args)
    assert os.path.basename(out) == "count_kernel_rmat-s20-ef16_kernel_trace.txt"
    lines = open(out).read().splitlines()
    assert any("rocprofv3 --kernel-trace --stats" in ln for ln in lines if ln.startswith("#"))
    body = [ln for ln in lines if not ln.startswith("#")]
    assert len(body) == 2  # the torch kernel is left out
    assert body[0].split()[-3:] == ["tc::count_kernel<1,", "false,", "int>"]
    calls, avg_us, min_us, max_us, total_ms = body[0].split()[:5]
    assert (int(calls), float(avg_us), float(min_us), float(max_us), float(total_ms)) == \
        (6, 2800.0, 2700.0, 2960.0, 16.8)


def test_pmc_summary_scales_by_the_calibration_copy(fake_root, monkeypatch):
    monkeypatch.setattr(bench, "count_source_digest", lambda: "feedbeef00000000")
    header = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # a 1 GiB copy reads back FETCH 524288 KiB (factor 2) and WRITE 1048576 KiB (factor 1)
    fetch = [[COPY, "FETCH_SIZE", 524288.0], [COPY, "FETCH_SIZE", 524288.0],
             [COPY, "FETCH_SIZE", 16.0],  # a small copy is not calibration
             [COUNT1, "FETCH_SIZE", 7000.0], [COUNT1, "FETCH_SIZE", 9000.0],
             [COUNT0, "FETCH_SIZE", 6000.0]]
    write = [[COPY, "WRITE_SIZE", 1048576.0], [COUNT1, "WRITE_SIZE", 10.0],
             [COUNT0, "WRITE_SIZE", 2.0]]
    _write_csv(str(fake_root / "pf" / "run_counter_collection.csv"), header, fetch)
    _write_csv(str(fake_root / "pw" / "run_counter_collection.csv"), header, write)
    args = argparse.Namespace(summarize_pmc=[str(fake_root / "pf"), str(fake_root / "pw")],
                              workload="rmat-s20-ef16", calibrate_copy_mib=1024,
                              profile_command=["a", "b"])
    rec = json.load(open(bench.summarize_pmc(args)))
    assert rec["source_digest"] == "feedbeef00000000"
    assert rec["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert rec["calibration"]["write_factor"] == pytest.approx(1.0)
    pv = rec["count_per_vertex"]
    assert pv["dispatches"] == 2
    assert pv["traffic_bytes_per_launch"] == pytest.approx(8000.0 * 1024 * 2 + 10.0 * 1024)
    assert rec["count_total_only"]["traffic_bytes_per_launch"] == pytest.approx(
        6000.0 * 1024 * 2 + 2.0 * 1024)
    assert rec["traffic_bytes_per_launch"] == pv["traffic_bytes_per_launch"]


def _profile_commands(path):
    if path.endswith(".json"):
        with open(path) as f:
            return [c for c in json.load(f)["commands"] if c.startswith("rocprofv3 -")]
    with open(path) as f:
        return [ln[1:].strip() for ln in f
                if ln.startswith("#") and ln[1:].strip().startswith("rocprofv3 -")]


def test_committed_profiles_name_commands_that_run_committed_files():
    prof = os.path.join(ROOT, "profiles")
    files = sorted(os.listdir(prof))
    assert any(f.endswith("_kernel_trace.txt") for f in files)
    for name in files:
        cmds = _profile_commands(os.path.join(prof, name))
        assert cmds, name
        for c in cmds:
            prog = c.split(" -- ", 1)[1].split()
            # the program follows the profiler directly and is the committed benchmark
            assert prog[0] == "python3" and "bench.py" in prog, (name, c)
            assert os.path.exists(os.path.join(ROOT, "bench.py"))
            workload = prog[prog.index("--workload") + 1]
            assert workload in bench.WORKLOADS, (name, workload)
            assert workload in name, (name, workload)


def test_cpu_baseline_whole_and_sampled():
    """The oracle baseline reports the whole-graph total when it counts every source, and a
    count time scaled from a uniform prefix of sources otherwise."""
    import graphgen
    import oracle
    s, d, n = graphgen.rmat(11, 16, 3)
    s, d = s.numpy(), d.numpy()
    T = oracle.triangles(n, s, d)
    m = int(oracle.clean(n, s, d)[0][-1]) // 2
    whole = bench.cpu_baseline("rmat-s11", s, d, n, m, frac=1.0)
    assert whole["total"] == T and whole["kind"] == "oracle" and whole["value"] > 0
    assert "scaled" not in whole["sample"]
    part = bench.cpu_baseline("rmat-s11", s, d, n, m, frac=0.25)
    assert part["total"] is None and part["value"] > 0
    assert f"below {n // 4} of {n}" in part["sample"]


def test_default_workload_is_scale24_with_a_stored_oracle_count():
    assert bench.DEFAULT_WORKLOAD == "rmat-s24-ef16"
    assert bench.WORKLOADS[bench.DEFAULT_WORKLOAD]["offset_bytes"] == 8
    g = bench.golden_for(bench.DEFAULT_WORKLOAD)
    assert g is not None and g["triangles"] > 2**32 and g["sum_t"] == 3 * g["triangles"]
    assert bench.golden_for("rmat-s20-ef16") is None


def test_calibration_copy_is_the_repeated_one():
    """A one-off larger copy (a clone of a bigger array) is not taken for the calibration
    copy, which the benchmark runs three times."""
    assert bench.calibration_copies([6.3e6, 5.243e5, 5.242e5, 5.244e5, 10.0]) == [
        5.243e5, 5.242e5, 5.244e5]
    assert bench.calibration_copies([7.0, 100.0, 99.0]) == [100.0, 99.0]
