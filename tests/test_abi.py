"""The C-ABI library loads and exports every function include/tc.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(tc_[a-z_0-9]+)\s*\(", text,
                                 flags=re.M)))


def declared_constants():
    return dict((k, int(v)) for k, v in re.findall(r"#define\s+(TC_[A-Z_]+)\s+(\d+)",
                                                   open(HEADER).read()))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ["tc_build_csr", "tc_orient", "tc_count", "tc_count_per_vertex",
                 "tc_count_batched", "tc_list_triangles", "tc_edge_support", "tc_ne_filter",
                 "tc_count_bfs", "tc_count_k4",
                 "tc_status_string", "tc_last_error", "tc_version"]:
        assert name in fns


def test_library_exports_every_declared_function():
    from paper_1909_02127_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_constants_match_header():
    from paper_1909_02127_amd import _lib
    for k, v in declared_constants().items():
        assert getattr(_lib, k) == v, k


def test_status_strings_and_version():
    from paper_1909_02127_amd import _lib
    assert _lib.status_string(0) == "TC_OK"
    assert _lib.status_string(4) == "TC_ERR_WORKSPACE"
    assert _lib.status_string(99) == "TC_ERR_UNKNOWN"
    assert _lib.tc_version() >= 100


def test_host_side_argument_errors_need_no_gpu():
    """Workspace queries and argument validation run on the host only."""
    from paper_1909_02127_amd import _lib
    assert _lib.tc_build_csr_workspace(1024, 8192) > 2 * 2 * 8192 * 8
    assert _lib.tc_orient_workspace(1024, 8192) > _lib.tc_orient_workspace(1024, 0) > 0
    assert _lib.tc_count_workspace(1024) > 0
    with pytest.raises(_lib.TcError) as e:
        _lib.tc_build_csr_workspace(-1, 10)
    assert e.value.status == _lib.TC_ERR_INVALID_ARG
    with pytest.raises(_lib.TcError) as e:
        _lib.tc_build_csr_workspace(10, 10, offset_bytes=2)
    assert e.value.status == _lib.TC_ERR_INVALID_ARG
    with pytest.raises(_lib.TcError) as e:
        _lib.tc_build_csr_workspace(1 << 31, 10)
    assert e.value.status == _lib.TC_ERR_UNSUPPORTED
    with pytest.raises(_lib.TcError) as e:
        _lib.tc_build_csr_workspace(10, (1 << 30) + 1, offset_bytes=4)
    assert e.value.status == _lib.TC_ERR_UNSUPPORTED
    assert _lib.tc_list_triangles_workspace(1024) > _lib.tc_list_triangles_workspace(0) > 0
    assert _lib.tc_edge_support_workspace(1024) > 0
    assert _lib.tc_ne_filter_workspace(1024, 64) > 0
    assert _lib.tc_count_bfs_workspace(1024, 1 << 20) > 16 * (1 << 20)
    with pytest.raises(_lib.TcError) as e:
        _lib.tc_ne_filter_workspace(10, 5000)
    assert e.value.status == _lib.TC_ERR_INVALID_ARG
    csr = _lib.tc_csr(10, 4, None, None)
    size = ctypes.c_size_t(0)
    st = _lib.LIB.tc_list_triangles(ctypes.byref(csr), None, -1, None, None, None,
                                    ctypes.byref(size), None)
    assert st == _lib.TC_ERR_INVALID_ARG and "capacity" in _lib.LIB.tc_last_error().decode()
    st = _lib.LIB.tc_orient(ctypes.byref(csr), 0, None, None, (1 << 40) + 1, None, None,
                            ctypes.byref(size), None)
    assert st == _lib.TC_ERR_UNSUPPORTED
    st = _lib.LIB.tc_orient(ctypes.byref(csr), 7, None, None, 0, None, None, ctypes.byref(size), None)
    assert st == _lib.TC_ERR_INVALID_ARG
    assert "order" in _lib.LIB.tc_last_error().decode()


def test_fresh_checkout_builds_without_a_library(tmp_path):
    """The build module must import before libtc.so exists; the binding must then refuse."""
    import shutil
    import subprocess
    import sys
    pkg = os.path.join(ROOT, "paper_1909_02127_amd")
    dst = tmp_path / "paper_1909_02127_amd"
    shutil.copytree(pkg, dst, ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__"))
    code = ("import paper_1909_02127_amd.build as b\n"
            "import paper_1909_02127_amd as tc\n"
            "try:\n    tc.triangle_count\nexcept ImportError:\n    print('refused')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "refused" in r.stdout
