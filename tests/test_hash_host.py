"""The LDS cuckoo hash of the count kernel, compiled as host code (no GPU).

A signed shift once turned slot indices negative for ids >= 207, sending LDS
accesses out of range; this test runs exactly the header the kernel includes.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_hash_indices_in_range(tmp_path):
    exe = tmp_path / "hash_range"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                    f"-I{ROOT}/paper_1909_02127_amd/csrc",
                    os.path.join(ROOT, "tests", "host", "hash_range.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "out_of_range=0" in r.stdout
    max_load = int(r.stdout.split("max_load=")[1])
    assert max_load <= 8
