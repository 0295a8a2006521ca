"""The C ABI library loads on a host without a GPU and exports every symbol
include/mibh.h declares; the pure host entry points behave as documented."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1204_2280_amd import build, mibh
    if not os.path.exists(mibh.LIB_PATH):
        build.build()
    return mibh.lib()


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mibh_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_host_only_entry_points(lib):
    from paper_1204_2280_amd import mibh
    p = mibh.default_params()
    assert (p.ncrit, p.group_cap, p.eps2, p.G, p.precision) == (16, 64, 0.0, 1.0, 0)
    b1 = mibh.workspace_bytes(1 << 20, p)
    b2 = mibh.workspace_bytes(1 << 22, p)
    assert 0 < b1 < b2 < 4 * 2 ** 30
    assert mibh.workspace_bytes(0, p) == 0
    assert mibh.workspace_bytes(1 << 31, p) == 0
    assert mibh.workspace_bytes(100, mibh.default_params(ncrit=65)) == 0
    assert mibh.workspace_bytes(100, mibh.default_params(group_cap=65)) == 0
    assert mibh.workspace_bytes(100, mibh.default_params(pc_cap=127)) == 0
    assert mibh.workspace_bytes(100, mibh.default_params(pc_cap=4096)) == 0
    assert lib.mibh_status_string(-5) == b"MIBH_EOVERFLOW"
    h = C.c_void_p()
    # invalid workspace pointer is rejected before any device call
    st = lib.mibh_create(C.byref(p), 100, None, 1 << 20, None, C.byref(h))
    assert st == -1 and b"workspace" in lib.mibh_last_error()
    st = lib.mibh_create(C.byref(p), 100, 256, 16, None, C.byref(h))
    assert st == -2
    assert lib.mibh_build_tree(None, None, None, 10) == -1
