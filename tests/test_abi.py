"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/soft.h, its structs have the layout the binding assumes,
and context creation without a device fails with an error code."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

from paper_2512_23037_amd import soft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "soft.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(soft.LIB_PATH):
        from paper_2512_23037_amd import build
        build.build()
    return soft.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(soft_[a-z_]+)\s*\(", text)))


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    assert sorted(soft.EXPORTS) == names
    for name in names:
        assert getattr(lib, name) is not None


def test_struct_layout_matches_binding(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "soft.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(soft_noise), sizeof(soft_counters),'
                   ' offsetof(soft_counters, support_hist), offsetof(soft_counters, max_norm_dev));'
                   ' printf("%zu\\n", offsetof(soft_counters, restarts));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [ctypes.sizeof(soft.soft_noise), ctypes.sizeof(soft.soft_counters),
                   soft.soft_counters.support_hist.offset, soft.soft_counters.max_norm_dev.offset,
                   soft.soft_counters.restarts.offset]


def test_header_compiles_as_c_and_cxx(tmp_path):
    for compiler, ext in (("gcc", "c"), ("g++", "cpp")):
        src = tmp_path / ("h." + ext)
        src.write_text('#include "soft.h"\nint main(void){soft_ctx *c = 0; (void)c; return SOFT_OK;}\n')
        subprocess.run([compiler, "-Wall", "-Werror", "-I", os.path.dirname(HEADER), "-c", str(src), "-o",
                        str(tmp_path / ("h_" + ext + ".o"))], check=True)


def test_create_without_device_reports_error(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    rc = lib.soft_create(ctypes.byref(h), 0)
    assert rc in (soft.SOFT_EDEVICE, soft.SOFT_EINVAL)
    assert not h.value
    assert lib.soft_last_error(None)
    lib.soft_destroy(None)  # NULL is allowed
