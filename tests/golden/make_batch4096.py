"""Writes batch4096_seed4.json: the oracle's counts for every graph of the packed
4096-graph batch (graphgen.batch_suite_spec(4096, seed=4): n log-uniform in
[2^8, 2^16], average degree uniform in [4, 64], Erdos-Renyi for even i and R-MAT
for odd i).

For each graph: n, m, the total T, and the first 16 hex digits of the SHA-256 of
its per-vertex counts t (uint64, little-endian), so a GPU run can check every
t(v) of every graph.  Calls only the oracle and the input generator; the graphs
are counted in a thread pool (the oracle releases the GIL).  Takes a few minutes
of CPU.  Run from the repository root:  python tests/golden/make_batch4096.py
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402

COUNT, SEED = 4096, 4
NAME = f"batch{COUNT}_seed{SEED}.json"


def t_digest(t: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(t, dtype="<u8").tobytes()).hexdigest()[:16]


def one(spec):
    s, d, n = graphgen.batch_graph(spec)
    s, d = s.numpy(), d.numpy()
    rp, col = oracle.clean(n, s, d)
    dp, dc = oracle.orient(rp, col, oracle.ORDER_DEGREE)
    total, t = oracle.count(dp, dc, per_vertex=True, threads=1)
    return {"i": spec.index, "kind": spec.kind, "n": n, "pairs": int(s.size),
            "m": int(dp[-1]), "triangles": int(total), "t_digest": t_digest(t)}


def main():
    t0 = time.time()
    specs = graphgen.batch_suite_spec(COUNT, seed=SEED)
    out = [None] * len(specs)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        for k, r in enumerate(ex.map(one, specs)):
            out[r["i"]] = r
            if (k + 1) % 512 == 0:
                print(f"{k + 1}/{len(specs)} graphs ({time.time() - t0:.0f}s)", flush=True)
    rec = {"generator": f"graphgen.batch_suite_spec({COUNT}, seed={SEED}) -> graphgen.batch_graph",
           "t_digest": "first 16 hex digits of sha256(t as little-endian uint64)",
           "sum_n": sum(r["n"] for r in out), "sum_m": sum(r["m"] for r in out),
           "sum_triangles": sum(r["triangles"] for r in out), "graphs": out}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), NAME)
    with open(path, "w") as f:
        json.dump(rec, f, separators=(",", ":"))
        f.write("\n")
    print("wrote", path, f"({time.time() - t0:.0f}s)")


if __name__ == "__main__":
    main()
