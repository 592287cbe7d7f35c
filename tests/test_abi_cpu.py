"""The C-ABI library loads and exports every entry point include/diffrt.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "diffrt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dr[A-Z]\w*)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["drSceneCreate", "drSceneUpdateVertices", "drRender", "drRenderBackward", "drSceneDestroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1904_12228_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libdiffrt.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == declared()
    # a pure host call: error strings
    lib.drGetErrorString.restype = ctypes.c_char_p
    assert lib.drGetErrorString(0) == b"success"
    assert lib.drGetErrorString(1) == b"invalid value"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1904_12228_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()
