"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad input in its host-side validation (which runs
before any HIP call).  No kernel is launched here."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bem.h")
PKG = os.path.join(ROOT, "paper_2003_12663_amd")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bem_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2003_12663_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libbem.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("bem_create", "bem_destroy", "bem_assemble", "bem_matvec", "bem_solve_gmres", "bem_eval_field",
                 "bem_trace_lines", "bem_streamer_integral", "bem_last_error"):
        assert name in fns


def test_library_exports_every_declared_symbol(lib):
    from paper_2003_12663_amd import _lib
    fns = declared_functions()
    missing = [f for f in fns if not hasattr(lib, f)]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == fns


def test_gfx950_code_object_present():
    from paper_2003_12663_amd import _lib
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_validation_before_any_hip_call(lib):
    from paper_2003_12663_amd import _lib
    ctx = ctypes.c_void_p()
    vert = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    tri = np.array([[0, 1, 2], [0, 1, 3]], dtype=np.int32)
    tb = np.zeros(2, dtype=np.int32)
    bodies = (_lib.Body * 1)(_lib.Body(0, 1.0, 1.0))

    def create(v, t, b, opt=None, nb=1, bd=bodies):
        return lib.bem_create(len(v), v.ctypes.data, len(t), t.ctypes.data, b.ctypes.data, nb,
                              ctypes.addressof(bd), ctypes.byref(opt) if opt else None, None, ctypes.byref(ctx))

    bad = tri.copy()
    bad[1, 2] = 9
    assert create(vert, bad, tb) == _lib.BEM_ERR_INVALID
    assert b"out of range" in lib.bem_last_error()
    v2 = vert.copy()
    v2[3, 2] = np.inf
    assert create(v2, tri, tb) == _lib.BEM_ERR_INVALID
    v3 = vert.copy()
    v3[2] = [2.0, 0.0, 0.0]                      # collinear with v0, v1
    assert create(v3, tri, tb) == _lib.BEM_ERR_DEGENERATE
    bb = np.array([0, 1], dtype=np.int32)
    assert create(vert, tri, bb) == _lib.BEM_ERR_INVALID
    opt = _lib.Options(0, 0.5, 100, 0)          # eta < 1
    assert create(vert, tri, tb, opt) == _lib.BEM_ERR_INVALID
    opt = _lib.Options(0, 6.0, 0, 0)            # restart 0
    assert create(vert, tri, tb, opt) == _lib.BEM_ERR_INVALID
    fl = (_lib.Body * 2)(_lib.Body(0, 1.0, 1.0), _lib.Body(1, 1.0, 1.0))   # floating body without panels
    assert create(vert, tri, tb, None, 2, fl) == _lib.BEM_ERR_INVALID
    assert ctx.value is None


def test_struct_layout_matches_header(tmp_path):
    """The ctypes structs of the binding have the sizes and field offsets of the C
    structs in include/bem.h (a probe compiled here with gcc)."""
    import subprocess
    from paper_2003_12663_amd import _lib
    structs = {"bem_body": _lib.Body, "bem_options": _lib.Options, "bem_solve_info": _lib.SolveInfo,
               "bem_trace_params": _lib.TraceParams}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bem.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_nodal_basis_validation_before_any_hip_call(lib):
    """The LINEAR basis: an unknown basis and vertices shared by two bodies are
    refused in host-side validation (every body kind and both constraint forms are
    accepted)."""
    from paper_2003_12663_amd import _lib
    ctx = ctypes.c_void_p()
    vert = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    tri = np.array([[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]], dtype=np.int32)

    def create(tb, bodies, opt):
        arr = (_lib.Body * len(bodies))(*[_lib.Body(*b) for b in bodies])
        tb = np.asarray(tb, dtype=np.int32)
        return lib.bem_create(len(vert), vert.ctypes.data, len(tri), tri.ctypes.data, tb.ctypes.data, len(bodies),
                              ctypes.addressof(arr), ctypes.byref(opt), None, ctypes.byref(ctx))

    one = [(0, 1.0, 1.0)]
    assert create([0, 0, 0, 0], one, _lib.Options(0, 6.0, 100, 1, 2)) == _lib.BEM_ERR_INVALID   # no such basis
    two = [(0, 1.0, 1.0), (0, 1.0, 1.0)]
    assert create([0, 0, 1, 1], two, _lib.Options(0, 6.0, 100, 1, 1)) == _lib.BEM_ERR_INVALID   # shared vertices
    assert b"shared" in lib.bem_last_error()
    assert ctx.value is None


def test_product_path_never_touches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.lower().replace("oracle-free", ""), f
