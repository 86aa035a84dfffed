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
