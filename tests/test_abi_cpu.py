"""The C-ABI library loads on the host and exports every entry point that
include/tn.h declares (no device calls)."""
import ctypes
import os
import re

import paper_2307_04890_amd as tn
from paper_2307_04890_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "tn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tn_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no Python binding"


def test_host_only_entry_points():
    assert tn.lib.tn_mlp_param_count() == 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1
    assert isinstance(tn.lib.tn_last_error(), bytes)
