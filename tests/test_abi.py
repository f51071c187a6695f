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


def test_noalloc_checks_arguments_before_any_work(lib):
    """wenotheta_rhs_noalloc rejects a grid whose divergence accumulator would exceed its
    fixed scratch buffer (WT_ERR_SCRATCH), WT_SIDES grids (no side table without a
    context) and bad arguments, all before any HIP call: this runs without a GPU.  The
    device pointers are placeholders that the checks never dereference."""
    f = lib.wenotheta_rhs_noalloc
    f.restype = ctypes.c_int
    G, P = ctypes.POINTER(binding.wt_grid), ctypes.POINTER(binding.wt_params)
    vp = ctypes.c_void_p
    f.argtypes = [G, P, vp, vp, ctypes.POINTER(ctypes.c_double), vp, vp, vp]
    fake = vp(0x1000)

    def call(grid, params=wt.Params(system=wt.WT_EULER), u=fake, L=fake):
        return f(ctypes.byref(grid.c_struct()), ctypes.byref(params.c_struct()), u, None, None, L,
                 None, None)

    def grid2(nx, ny, bc=wt.WT_TRANSMISSIVE):
        return wt.Grid(n=(nx, ny), lo=(0.0, 0.0), hi=(1.0, 1.0), bc=(bc, bc))

    # 2D Euler: 4 * nx * ny doubles of divergence; the buffer holds 8388096
    assert call(grid2(1449, 1449)) == binding.WT_ERR_SCRATCH
    assert call(grid2(2048, 1024)) == binding.WT_ERR_SCRATCH
    g3 = wt.Grid(n=(128, 128, 128), lo=(0.0,) * 3, hi=(1.0,) * 3, bc=(0, 0, 0))
    assert call(g3) == binding.WT_ERR_SCRATCH
    assert call(grid2(64, 64, bc=wt.WT_SIDES)) == binding.WT_ERR_UNSUPPORTED
    assert call(grid2(5, 64)) == binding.WT_ERR_ARG                 # fewer than 6 points
    assert call(grid2(64, 64), u=None) == binding.WT_ERR_ARG
    assert call(grid2(64, 64), L=None) == binding.WT_ERR_ARG
    assert call(grid2(64, 64), params=wt.Params(system=wt.WT_EULER, cfl=0.0)) == binding.WT_ERR_ARG
    msg = lib.wenotheta_status_string
    msg.restype = ctypes.c_char_p
    msg.argtypes = [ctypes.c_int32]
    assert b"scratch" in msg(binding.WT_ERR_SCRATCH)
