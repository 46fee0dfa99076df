"""The C-ABI library loads on a host without a GPU and exports every entry point that
include/wcc.h declares (no compute calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wcc.h")
LIB = os.path.join(ROOT, "paper_2509_02590_amd", "_build", "libwcc.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(wcc_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("wcc_run", "wcc_mincut_split", "wcc_mincut_split_batch", "wcc_cluster_csr",
                 "wcc_strerror", "wcc_threshold", "wcc_default_params"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_helpers():
    import oracle
    from paper_2509_02590_amd import _lib
    assert _lib.lib.wcc_abi_version() == 1
    for crit in ("log10", "log2", "sqrt"):
        for n in list(range(1, 3000)) + [10**6 - 1, 10**6, 10**6 + 1, 2**24]:
            assert _lib.threshold(n, crit) == oracle.threshold(n, crit)
    assert _lib.threshold(100, "linear", 3, 10) == oracle.threshold(100, "linear", 3, 10)
    assert _lib.lib.wcc_strerror(-2).decode().startswith("malformed")
