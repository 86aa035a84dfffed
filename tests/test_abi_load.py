"""The C-ABI library loads and exports every symbol include/gicp.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gicp.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gicp_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2403_12550_amd import _abi, build
    if not os.path.exists(_abi.LIB_PATH):
        build.build()
    return _abi.LIB_PATH


def test_header_declares_the_calls():
    names = _declared()
    for n in ["gicp_create", "gicp_destroy", "gicp_knn", "gicp_covariances", "gicp_map_build",
              "gicp_register", "gicp_register_pair", "gicp_strerror"]:
        assert n in names


def test_every_declared_symbol_is_exported(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header(libpath):
    from paper_2403_12550_amd import _abi
    _abi.load(libpath)
    assert set(_declared()) <= set(_abi.SIGNATURES)


def test_host_only_calls(libpath):
    from paper_2403_12550_amd import _abi
    lib = _abi.load(libpath)
    assert lib.gicp_strerror(0) == b"ok"
    assert lib.gicp_strerror(4).startswith(b"degenerate")
    p = _abi.Params()
    lib.gicp_params_default(ctypes.byref(p))
    assert (p.k, p.max_it, p.reg_mode) == (20, 30, 1)
    assert abs(p.eps - 1e-3) < 1e-9 and abs(p.r_max - 0.1) < 1e-7
    # argument validation happens before any device call
    assert lib.gicp_create(None, 0) == _abi.GICP_E_ARG
    assert lib.gicp_covariances(None, None, 0, 20, 0.0, 1, 1e-3, None, None) == _abi.GICP_E_ARG


def test_batch_structs_match_the_header_layout():
    """The batched binding fills gicp_problem and gicp_stats through numpy
    structured arrays; their field offsets must be the ctypes (C) ones."""
    import ctypes as C

    import paper_2403_12550_amd as g
    assert g._PROBLEM_DT.itemsize == C.sizeof(g.Problem)
    assert g._STATS_DT.itemsize == C.sizeof(g.Stats)
    for name, _ in g.Problem._fields_:
        assert g._PROBLEM_DT.fields[name][1] == getattr(g.Problem, name).offset, name
    for name, _ in g.Stats._fields_:
        assert g._STATS_DT.fields[name][1] == getattr(g.Stats, name).offset, name


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; N > 1 exits with a message before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
