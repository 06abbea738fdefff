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


# binding class -> C typedef in include/vx.h
_STRUCTS = {"Col": "vx_col", "Stats": "vx_stats", "LinkCalib": "vx_link_calib", "JoinRows": "vx_join_rows",
            "BuildDesc": "vx_build_desc", "Agg": "vx_agg", "ProbeDesc": "vx_probe_desc", "StarDim": "vx_star_dim",
            "GroupRow": "vx_group_row", "StarJoin": "vx_star_join", "BatchJoin": "vx_batch_join",
            "PartOpts": "vx_part_opts", "SortDesc": "vx_sort_desc", "PartitionedJoin": "vx_partitioned_join",
            "RadixJoin": "vx_radix_join", "JoinDesc": "vx_join_desc", "JoinOut": "vx_join_out",
            "PartitionDesc": "vx_partition_desc", "PartitionOut": "vx_partition_out"}


def test_struct_layouts_match_header(tmp_path):
    """Every struct of the binding has the size and field offsets the C compiler gives the
    header's typedef (a C program built with gcc prints them)."""
    import subprocess
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "vx.h"', "int main(void) {"]
    want = {}
    for py, c in _STRUCTS.items():
        cls = getattr(vx, py)
        lines.append(f'  printf("{py} %zu\\n", sizeof({c}));')
        want[py] = ctypes.sizeof(cls)
        for f in cls._fields_:
            lines.append(f'  printf("{py}.{f[0]} %zu\\n", offsetof({c}, {f[0]}));')
            want[f"{py}.{f[0]}"] = getattr(cls, f[0]).offset
    lines.append("  return 0;\n}")
    (tmp_path / "layout.c").write_text("\n".join(lines))
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(tmp_path / "layout.c"), "-o",
                    str(tmp_path / "layout")], check=True, capture_output=True)
    out = subprocess.run([str(tmp_path / "layout")], check=True, capture_output=True, text=True).stdout
    got = {k: int(v) for k, v in (line.split() for line in out.splitlines())}
    assert got == want
