"""The C-ABI library loads and exports every symbol the header declares
(CPU only: no device calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(sg_\w+)\s*\(", text))
    return names


def test_header_declares_entry_points():
    names = _declared()
    assert {"sg_create", "sg_simulate", "sg_batch_step", "sg_autotune"} <= names


def test_library_exports_every_declared_symbol():
    from paper_2507_01152_amd import sonosim
    if not os.path.exists(sonosim.LIB_PATH):
        pytest.fail("libsonosim.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(sonosim.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    assert set(_declared()) <= set(sonosim.SYMBOLS) | {"sg_last_error"}


def test_version_and_error_string_without_device():
    from paper_2507_01152_amd import sonosim
    lib = sonosim.load()
    assert lib.sg_version() == 100
    assert isinstance(lib.sg_last_error(), bytes)
