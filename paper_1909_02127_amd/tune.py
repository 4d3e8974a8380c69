"""Autotuner for the count kernels' launch parameters (tc_tune).

It times a grid of candidates -- the wave/workgroup split threshold on d+(u),
the probe structure (LDS cuckoo table or sorted binary search), and the number
of persistent workgroups per compute unit -- with HIP events on the current
stream and keeps the fastest.  Results are cached in a JSON file keyed by the
device name and a caller-supplied workload class.  Tuning changes only the
speed: every candidate computes the same counts.
"""
from __future__ import annotations

import json
import os
from pathlib import Path

import torch

from ._lib import TC_PROBE_AUTO, TC_PROBE_SORTED

DEFAULT_CANDIDATES = [
    {"small_max": s, "probe": p, "blocks_per_cu": b}
    for s in (16, 32, 64, 96)
    for p in (TC_PROBE_AUTO, TC_PROBE_SORTED)
    for b in (0, 4)
] + [
    # the equal-work quantum of split sources, at the default split and probe
    {"small_max": 96, "probe": TC_PROBE_AUTO, "blocks_per_cu": 0, "split_log2": q}
    for q in (14, 17, -1)
]


def cache_path() -> Path:
    return Path(os.environ.get("TC_TUNE_CACHE", Path.home() / ".cache" / "tc_tune.json"))


def _load_cache() -> dict:
    p = cache_path()
    if p.exists():
        try:
            return json.loads(p.read_text())
        except (OSError, ValueError):
            return {}
    return {}


def _store_cache(cache: dict) -> None:
    p = cache_path()
    try:
        p.parent.mkdir(parents=True, exist_ok=True)
        tmp = p.with_suffix(".tmp")
        tmp.write_text(json.dumps(cache, indent=1))
        os.replace(tmp, p)
    except OSError:
        pass


def time_ms(run, reps: int = 3) -> float:
    """Median milliseconds of `run()` over `reps` launches, after one warm-up."""
    run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def autotune(run_with, workload_class: str, *, candidates=None, reps: int = 3,
             use_cache: bool = True, timer=None, device_name: str | None = None
             ) -> tuple[dict, list]:
    """run_with(tune_dict) enqueues one count.  Returns (best tune, [(tune, ms), ...]).
    `timer(run, reps)` measures one candidate (default: HIP events, time_ms); the cache key
    is the device name and the caller's workload class."""
    dev = device_name if device_name is not None else torch.cuda.get_device_name()
    key = f"{dev}|{workload_class}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key]["tune"], cache[key].get("table", [])
    timer = timer or time_ms
    table = []
    for cand in candidates or DEFAULT_CANDIDATES:
        table.append((cand, timer(lambda c=cand: run_with(c), reps)))
    best = min(table, key=lambda x: x[1])[0]
    if use_cache:
        cache[key] = {"tune": best, "table": table}
        _store_cache(cache)
    return best, table
