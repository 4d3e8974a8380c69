"""Writes rmat_s24_ef16_seed24.json: the oracle's counts for R-MAT scale 24, edge
factor 16, seed 24 (268,435,456 raw pairs, int64 offsets in the GPU run).

The whole per-vertex array t (16.7M uint64) is too large to store, so the file
keeps the total T, the SHA-256 of t as little-endian uint64 bytes (so a GPU run
can check every t(v) at once), sum(t) (= 3T), and t(v) itself for a sample of
vertices: the 64 with the largest t and 512 drawn uniformly from those with
t > 0.  It also keeps the wedge count of the degree-ordered DAG and the largest
out-degree, which size the benchmark's roofline.

Calls only the oracle and the input generator.  Takes several minutes of CPU
(the oracle is single-threaded except for its count).  Run from the repository
root:  python tests/golden/make_rmat_s24.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen  # noqa: E402
import oracle  # noqa: E402

SCALE, EF, SEED = 24, 16, 24
NAME = f"rmat_s{SCALE}_ef{EF}_seed{SEED}.json"


def main():
    t0 = time.time()
    s, d, n = graphgen.rmat(SCALE, EF, SEED)
    s, d = s.numpy(), d.numpy()
    print(f"generated {s.size} pairs ({time.time() - t0:.0f}s)", flush=True)
    rp, col = oracle.clean(n, s, d)
    print(f"clean: 2m = {rp[-1]} ({time.time() - t0:.0f}s)", flush=True)
    dp, dc = oracle.orient(rp, col, oracle.ORDER_DEGREE)
    del col
    dplus = np.diff(dp)
    wedges = int(dplus[dc.astype(np.int64)].sum())
    print(f"orient: m = {dp[-1]} ({time.time() - t0:.0f}s)", flush=True)
    total, t = oracle.count(dp, dc, per_vertex=True)
    print(f"count: T = {total} ({time.time() - t0:.0f}s)", flush=True)
    t = np.ascontiguousarray(t, dtype="<u8")
    top = np.argsort(-t.astype(np.int64), kind="stable")[:64]
    rng = np.random.default_rng(SEED)
    nz = np.flatnonzero(t)
    rand = np.sort(rng.choice(nz, size=min(512, nz.size), replace=False))
    sample = sorted(set(int(v) for v in top) | set(int(v) for v in rand))
    out = {
        "generator": f"graphgen.rmat({SCALE}, {EF}, {SEED})",
        "n": int(n), "raw_pairs": int(s.size), "m": int(dp[-1]), "nnz": int(rp[-1]),
        "triangles": int(total), "sum_t": int(t.sum(dtype=np.uint64)),
        "t_sha256": hashlib.sha256(t.tobytes()).hexdigest(),
        "t_sample": {str(v): int(t[v]) for v in sample},
        "degree_order": {"wedges": wedges, "max_out_degree": int(dplus.max()),
                         "max_degree": int(np.diff(rp).max())},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), NAME)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path, f"({time.time() - t0:.0f}s)")


if __name__ == "__main__":
    main()
