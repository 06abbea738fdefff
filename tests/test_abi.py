"""The C-ABI library loads and exports every entry point include/vx.h declares (CPU only)."""
import ctypes
import os
import re

import paper_2502_09541_amd as vx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "vx.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(vx_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_boundary():
    names = declared_functions()
    for n in ("vx_build", "vx_probe_stream", "vx_join_agg", "vx_partition", "vx_ctx_create",
              "vx_last_error"):
        assert n in names
    assert set(names) == set(vx.EXPORTS)


def test_library_exports_every_symbol():
    lib = ctypes.CDLL(vx.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_last_error_without_gpu():
    L = vx.lib()
    assert isinstance(L.vx_last_error(), bytes)


def test_struct_sizes_match_c_layout():
    # sizes computed from the header's field order with natural alignment (x86-64)
    assert ctypes.sizeof(vx.Col) == 16
    assert ctypes.sizeof(vx.Agg) == 72
    assert ctypes.sizeof(vx.BuildDesc) == 48
    assert ctypes.sizeof(vx.ProbeDesc) == 72
    assert ctypes.sizeof(vx.GroupRow) == 48
