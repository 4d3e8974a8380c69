"""The autotuner's selection and cache logic on the CPU, with a stand-in timer (no GPU):
it times every candidate once, keeps the fastest, stores the table under the device name
and workload class, and answers from the cache without timing again."""
import json

from paper_1909_02127_amd import tune


def _fake_timer(costs, calls):
    def timer(run, reps):
        cand = run()
        calls.append(cand)
        return costs(cand)
    return timer


def test_picks_the_fastest_candidate_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("TC_TUNE_CACHE", str(tmp_path / "tune.json"))
    cands = tune.DEFAULT_CANDIDATES
    # cost: prefers split 64, the cuckoo probe, occupancy grid and the 2^17 quantum
    def costs(c):
        return (abs(c["small_max"] - 64) + 5 * c["probe"] + c["blocks_per_cu"]
                + (0 if c.get("split_log2") == 17 else 1))
    calls = []
    best, table = tune.autotune(lambda c: c, "wl", timer=_fake_timer(costs, calls),
                                device_name="dev0")
    assert len(calls) == len(cands) == len(table)
    assert best == min(cands, key=costs)
    assert [t for t, _ in table] == cands
    stored = json.loads((tmp_path / "tune.json").read_text())
    assert stored["dev0|wl"]["tune"] == best
    # a second call answers from the cache without timing
    calls2 = []
    best2, _ = tune.autotune(lambda c: c, "wl", timer=_fake_timer(costs, calls2),
                             device_name="dev0")
    assert best2 == best and calls2 == []
    # another device or workload class is tuned afresh
    calls3 = []
    tune.autotune(lambda c: c, "wl", timer=_fake_timer(costs, calls3), device_name="dev1")
    assert len(calls3) == len(cands)


def test_candidates_cover_split_probe_occupancy_and_quantum():
    keys = {k for c in tune.DEFAULT_CANDIDATES for k in c}
    assert {"small_max", "probe", "blocks_per_cu", "split_log2"} <= keys
    from paper_1909_02127_amd import _lib
    for c in tune.DEFAULT_CANDIDATES:
        _lib.make_tune(**c)  # every candidate is a valid tc_tune


def test_no_cache_means_no_file(tmp_path, monkeypatch):
    monkeypatch.setenv("TC_TUNE_CACHE", str(tmp_path / "tune.json"))
    tune.autotune(lambda c: c, "wl", timer=lambda run, reps: 1.0, device_name="d",
                  use_cache=False, candidates=[{"small_max": 16}])
    assert not (tmp_path / "tune.json").exists()
