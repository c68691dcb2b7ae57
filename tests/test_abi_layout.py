"""The Python binding's ctypes structures against the C header: a small C
program compiled with the host compiler prints sizeof and offsetof of every
field of the public structs, which must equal the ctypes layout field by
field (a field added to the header but not to the binding, or in another
place, fails here rather than as garbage parameters on the device)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2605_00619_amd import afe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "afe_mesh": afe._Mesh,
    "afe_params": afe._Params,
    "afe_info": afe._Info,
    "afe_step_report": afe._Report,
    "afe_launch_shape": afe._Shape,
    "afe_batch_report": afe._BatchReport,
}


def _c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "afe.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'    printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {}
    for line in out.splitlines():
        name, field, value = line.split()
        layout[(name, field)] = int(value)
    return layout


def test_ctypes_structs_match_the_header(tmp_path):
    layout = _c_layout(tmp_path)
    for name, cls in STRUCTS.items():
        assert ctypes.sizeof(cls) == layout[(name, "sizeof")], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == layout[(name, field)], (name, field)
