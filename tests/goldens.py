"""Reader for the hand-checked fixtures in tests/golden/*.txt."""
from __future__ import annotations

import glob
import os
from dataclasses import dataclass

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@dataclass
class Fixture:
    name: str
    why: str
    n: int
    triangles: int
    per_vertex: np.ndarray
    src: np.ndarray
    dst: np.ndarray
    triangle_sets: list  # sorted list of sorted vertex triples, hand-derived from `why`


def load(path: str) -> Fixture:
    meta, s, d = {}, [], []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                k, _, v = line[1:].partition(":")
                meta[k.strip()] = v.strip()
                continue
            a, b = line.split()
            s.append(int(a))
            d.append(int(b))
    sets = sorted(tuple(sorted(int(x) for x in t.split(",")))
                  for t in meta.get("triangle_sets", "").split())
    return Fixture(meta["name"], meta["why"], int(meta["n"]), int(meta["triangles"]),
                   np.array([int(x) for x in meta["per_vertex"].split()], dtype=np.uint64),
                   np.array(s, dtype=np.int32), np.array(d, dtype=np.int32), sets)


def all_fixtures() -> list[Fixture]:
    return [load(p) for p in sorted(glob.glob(os.path.join(GOLDEN_DIR, "*.txt")))]
