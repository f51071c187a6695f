"""The C-ABI library loads and exports every symbol include/wenotheta.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1504_00731_amd as wt
from paper_1504_00731_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wenotheta.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wenotheta_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1504_00731_amd import build
        build.build()
    return ctypes.CDLL(binding.LIB_PATH)


def test_header_declares_the_abi():
    names = declared_functions()
    assert {"wenotheta_rhs", "wenotheta_step", "wenotheta_solve"} <= set(names)
    assert set(names) == set(binding.EXPORTED)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    f = lib.wenotheta_status_string
    f.restype = ctypes.c_char_p
    f.argtypes = [ctypes.c_int32]
    assert f(0) == b"ok"
    assert b"non-physical" in f(3)
    assert f(99) == b"unknown status"


def test_struct_layout_matches_header(tmp_path):
    """Sizes and field offsets of the binding's structures equal those a C compiler
    gives the header's (compiled here with gcc against include/wenotheta.h)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    fields = {"wt_grid": [f[0] for f in binding.wt_grid._fields_],
              "wt_params": [f[0] for f in binding.wt_params._fields_],
              "wt_side": [f[0] for f in binding.wt_side._fields_]}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "wenotheta.h"', "int main(void) {"]
    for st, names in fields.items():
        src.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for n in names:
            src.append(f'printf("{st} {n} %zu\\n", offsetof({st}, {n}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st, names in fields.items():
        cls = getattr(binding, st)
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for n in names:
            assert got[(st, n)] == getattr(cls, n).offset, (st, n)


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(binding, "_LIB", None)
    monkeypatch.setattr(binding, "LIB_PATH", "/nonexistent/libwenotheta.so")
    with pytest.raises(binding.LibraryMissing):
        wt.Context(0)
