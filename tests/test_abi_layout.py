"""CPU check that the ctypes mirrors in the binding have the sizes and field
offsets of the C structs in include/*.h: a small C program compiled with the
host compiler prints sizeof / offsetof for every field the binding names."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# C struct name -> binding class name
STRUCTS = {
    "atlas_mesh_desc": "MeshDesc", "atlas_mesh_info": "MeshInfo",
    "atlas_mesh_layout": "Layout", "atlas_launch": "Launch",
    "atlas_work_item": "WorkItem", "atlas_batch_config": "BatchConfig",
    "atlas_batch_info": "BatchInfo", "atlas_serve_config": "ServeConfig",
    "atlas_request": "Request", "atlas_result": "Result",
    "atlas_serve_stats": "ServeStats", "atlas_remap_info": "RemapInfo",
}
# binding field names that differ from the C names
RENAMED = {("WorkItem", "in_"): "in", ("Request", "in_"): "in"}


@pytest.fixture(scope="module")
def layouts(tmp_path_factory):
    from paper_1908_06091_amd import _abi
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no host C compiler or HIP headers")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "atlas_nabla.h"',
             '#include "atlas_batch.h"', '#include "atlas_serve.h"', '#include "atlas_remap.h"',
             'int main(void) {']
    for cname, pyname in STRUCTS.items():
        lines.append(f'  printf("{pyname} size %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(_abi, pyname)._fields_:
            cf = RENAMED.get((pyname, fname), fname)
            lines.append(f'  printf("{pyname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ['  return 0;', '}']
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c11", "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include",
                    "-I/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        cls, field, val = line.split()
        got[(cls, field)] = int(val)
    return _abi, got


@pytest.mark.parametrize("pyname", sorted(STRUCTS.values()))
def test_ctypes_mirror_matches_header(layouts, pyname):
    _abi, got = layouts
    cls = getattr(_abi, pyname)
    assert ctypes.sizeof(cls) == got[(pyname, "size")], pyname
    for fname, _ in cls._fields_:
        assert getattr(cls, fname).offset == got[(pyname, fname)], (pyname, fname)
