"""The binding's mirrors of the C structs in include/awg.h have the header's
size and field offsets: a small C program compiled against the header prints
them (gcc, host only) and each ctypes / numpy layout is compared field by field."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import paper_2403_15582_amd as awg
from paper_2403_15582_amd.abi_types import TONE_DTYPE

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MIRRORS = {name: getattr(awg, name) for name in (
    "awg_plan_params", "awg_plan_info", "awg_kernel_stat", "awg_server_params", "awg_job",
    "awg_chunk_event", "awg_server_stats", "awg_retune", "awg_amp_ramp")}


def _c_layouts(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "awg.h"', "int main(void) {"]
    structs = dict(MIRRORS)
    for name, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines.append('printf("awg_tone size %zu\\n", sizeof(awg_tone));')
    for f in TONE_DTYPE.names:
        lines.append('printf("awg_tone %s %%zu\\n", offsetof(awg_tone, %s));' % (f, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-Wall", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    return got


def test_struct_layouts_match_the_header(tmp_path):
    c = _c_layouts(tmp_path)
    for name, cls in MIRRORS.items():
        assert c[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert c[(name, f)] == getattr(cls, f).offset, (name, f)
    assert c[("awg_tone", "size")] == TONE_DTYPE.itemsize
    for f in TONE_DTYPE.names:
        assert c[("awg_tone", f)] == TONE_DTYPE.fields[f][1], f
    # every field of the C struct is mirrored: the last offset plus its size is the size
    last = TONE_DTYPE.names[-1]
    assert TONE_DTYPE.fields[last][1] + TONE_DTYPE.fields[last][0].itemsize == TONE_DTYPE.itemsize


def test_plain_c_consumer_compiles_and_links(tmp_path):
    """tests/c/abi_consumer.c builds as strict C99 against include/awg.h and links
    libawg.so (the GPU test runs it)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("build_consumer", os.path.join(ROOT, "tests", "c", "build_consumer.py"))
    bc = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bc)
    exe = bc.build(str(tmp_path / "abi_consumer"))
    out = subprocess.run(["ldd", exe], check=True, capture_output=True, text=True).stdout
    assert "libawg.so" in out and "not found" not in out
