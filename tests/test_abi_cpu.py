"""The C-ABI library loads on a machine without a GPU and exports every entry
point the headers under include/ declare (no compute is launched here)."""
import ctypes
import os
import re

import pytest

from paper_2512_12151_amd import bfal

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def declared():
    src = "".join(open(os.path.join(INCLUDE, f)).read() for f in sorted(os.listdir(INCLUDE)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_binding_surface():
    names = declared()
    assert names == sorted(bfal.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(bfal.LIB_PATH):
        pytest.skip("libbfal.so not built")
    L = ctypes.CDLL(bfal.LIB_PATH)
    for n in declared():
        assert hasattr(L, n), n
    bfal.lib()   # prototypes bind


def test_footprint_is_host_only_and_monotone():
    if not os.path.exists(bfal.LIB_PATH):
        pytest.skip("libbfal.so not built")
    a = bfal.footprint_bytes(250, 768, 65)
    b = bfal.footprint_bytes(26620, 120000, 20000)
    assert 0 < a < b
    with pytest.raises(bfal.BfalError):
        bfal.footprint_bytes(0, 10, 1)
