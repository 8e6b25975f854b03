"""The C-ABI library loads and exports every entry point include/mgfr.h declares (no GPU:
only symbol lookups, no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgfr.h")
LIB = os.path.join(ROOT, "paper_1110_1379_amd", "libmgfr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgf?r?_[a-z0-9_]+)\s*\(", text)) - {"mgfr_ctx"})


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1110_1379_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_solver_entry_points():
    names = declared_functions()
    for required in ("mgfr_create", "mgfr_destroy", "mgfr_last_error", "mg_fr_solve", "mgfr_residual"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in mgfr.h but not exported"


def test_python_binding_names_match_the_header():
    from paper_1110_1379_amd import mgfr
    assert set(mgfr.exported_symbols()) <= set(declared_functions())
    for name in declared_functions():
        assert name in mgfr.exported_symbols(), f"{name} has no binding"


def test_struct_layouts_match_the_header():
    """ctypes mirrors of mgfr_params / mgfr_opts have the C sizes (checked with gcc)."""
    import subprocess
    import tempfile
    from paper_1110_1379_amd import mgfr
    src = ('#include "mgfr.h"\n#include <stdio.h>\nint main(){printf("%zu %zu %zu %zu\\n", '
           'sizeof(mgfr_params), sizeof(mgfr_opts), sizeof(mgfr_stats), sizeof(mgfr_patch));return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "s")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        a, b, c, d = map(int, subprocess.check_output([exe]).split())
    assert ctypes.sizeof(mgfr.mgfr_params) == a
    assert ctypes.sizeof(mgfr.mgfr_opts) == b
    assert ctypes.sizeof(mgfr.mgfr_stats) == c
    assert ctypes.sizeof(mgfr.mgfr_patch) == d
