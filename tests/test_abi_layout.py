"""The ctypes structures of the Python binding match the C structures of include/dmrg.h: a small C
program, compiled with the host compiler against the header, prints every structure's size and each
field's offset, and the binding's ctypes classes must agree field by field (CPU only)."""
import json
import os
import shutil
import subprocess

import pytest

lib_mod = pytest.importorskip("paper_2001_04890_amd")
from paper_2001_04890_amd import binding  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = {"Problem": "dmrg_problem", "OpDesc": "dmrg_op", "BlockDesc": "dmrg_block", "BuildOpts": "dmrg_build_opts",
         "DavOpts": "dmrg_dav_opts", "DavResult": "dmrg_dav_result", "DavBatchResult": "dmrg_dav_batch_result",
         "SweepOpts": "dmrg_sweep_opts", "SweepResult": "dmrg_sweep_result"}


def c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dmrg.h"', "int main(void) {", 'printf("{");']
    first = True
    for py, c in PAIRS.items():
        cls = getattr(binding, py)
        sep = "" if first else ","
        first = False
        lines.append(f'printf("{sep}\\"{py}\\": {{\\"size\\": %zu", sizeof({c}));')
        for name, _ in cls._fields_:
            lines.append(f'printf(", \\"{name}\\": %zu", offsetof({c}, {name}));')
        lines.append('printf("}");')
    lines += ['printf("}\\n");', "return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    return json.loads(subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout)


def test_ctypes_structures_match_the_header(tmp_path):
    layout = c_layout(tmp_path)
    for py in PAIRS:
        cls = getattr(binding, py)
        got = layout[py]
        assert binding.C.sizeof(cls) == got["size"], (py, binding.C.sizeof(cls), got["size"])
        for name, _ in cls._fields_:
            assert getattr(cls, name).offset == got[name], (py, name, getattr(cls, name).offset, got[name])
