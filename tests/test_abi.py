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
