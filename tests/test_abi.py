"""The C-ABI library loads and exports every entry point include/twg.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1903_07441_amd", "libtwg.so")
HDR = os.path.join(ROOT, "include", "twg.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*((?:twg|hpf)_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("twg_ctx_create", "twg_ctx_destroy", "twg_last_error", "twg_rasterize",
                 "hpf_relax", "hpf_descend", "hpf_sweeps", "hpf_residual", "hpf_index_matrix"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtwg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.twg_version() >= 100


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtwg.so not built")
def test_binding_exports_match_header():
    from paper_1903_07441_amd import twg
    assert sorted(twg.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libtwg.so not built")
def test_host_side_argument_checks_without_gpu():
    # twg_last_error on a NULL context and twg_ctx_create with a NULL out
    # pointer are answered on the host before any device call.
    lib = ctypes.CDLL(LIB)
    lib.twg_ctx_create.restype = ctypes.c_int32
    lib.twg_ctx_create.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    assert lib.twg_ctx_create(None, 0) == -1
    lib.twg_last_error.restype = ctypes.c_char_p
    lib.twg_last_error.argtypes = [ctypes.c_void_p]
    assert lib.twg_last_error(None) == b"null context"


def test_oracle_is_not_reachable_from_the_product():
    # the product path never imports or links the oracle
    pkg = os.path.join(ROOT, "paper_1903_07441_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                for bad in ("import oracle", "from oracle", "liboracle", "twg_oracle", "orc_"):
                    assert bad not in text, (fn, bad)
