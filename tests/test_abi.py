"""The C-ABI library loads and exports every function include/glnk.h declares
(no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "glnk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(gl_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libpath():
    from paper_1204_5125_amd import build, glnk
    if not os.path.exists(glnk.LIB_PATH):
        build.build()
    return glnk.LIB_PATH


def test_header_declares_boundary():
    names = declared_functions()
    for f in ("gl_residual", "gl_jacobian_apply", "gl_precond_setup", "gl_precond_apply",
              "gl_jacobian_solve", "gl_newton_solve"):
        assert f in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing


def test_binding_covers_header():
    from paper_1204_5125_amd import glnk
    assert sorted(glnk.EXPORTED_SYMBOLS) == declared_functions()


def test_status_strings(libpath):
    lib = ctypes.CDLL(libpath)
    lib.gl_status_string.restype = ctypes.c_char_p
    assert lib.gl_status_string(0) == b"ok"
    assert lib.gl_status_string(7) == b"singular preconditioner matrix"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1204_5125_amd import glnk
    monkeypatch.setattr(glnk, "_lib", None)
    monkeypatch.setattr(glnk, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        glnk.lib()


# ctypes mirror of each C struct of the header
STRUCTS = {"gl_grid_desc": "GridDesc", "gl_amg_opts": "AmgOpts", "gl_krylov_opts": "KrylovOpts",
           "gl_krylov_info": "KrylovInfo", "gl_newton_opts": "NewtonOpts", "gl_tiles": "Tiles",
           "gl_adam_opts": "AdamOpts", "gl_newton_info": "NewtonInfo", "gl_simplicial_desc": "SimplicialDesc"}


def test_binding_struct_layouts_match_header(tmp_path):
    """Size and every field offset of the binding's ctypes structures equal
    what the C compiler lays out from include/glnk.h."""
    import shutil
    import subprocess

    from paper_1204_5125_amd import glnk
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "glnk.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(glnk, pyname)
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, pyname in STRUCTS.items():
        cls = getattr(glnk, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])
