"""Writes er1024_8192.json: oracle counts for G(n=1024, m=8192), seeds 0-9.

Calls only the oracle and the input generator.  The test suite re-derives every
stored value with trace(A^3)/6 and diag(A^3)/2, independently of the oracle.
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402


def main():
    out = {"generator": "graphgen.erdos_renyi(1024, 8192, seed)", "graphs": {}}
    for seed in range(10):
        s, d, n = graphgen.erdos_renyi(1024, 8192, seed)
        total, per = oracle.triangles(n, s.numpy(), d.numpy(), per_vertex=True)
        out["graphs"][str(seed)] = {"n": n, "m": 8192, "triangles": total,
                                    "per_vertex": [int(x) for x in per]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "er1024_8192.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
