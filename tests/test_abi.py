"""The C ABI library loads without a GPU and exports every entry point that
include/*.h declares (no compute calls)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2405_17696_amd", "libhelm.so")


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", txt, flags=re.M):
            name = m.group(1)
            if name.startswith(("helm_", "cnn_", "fwi_")):
                names.append(name)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("helm_setup", "helm_matvec", "helm_solve", "helm_destroy", "helm_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_header():
    from paper_2405_17696_amd import _lib
    missing = [n for n in declared_functions() if n not in _lib.SIGNATURES]
    assert not missing, missing
    lib = _lib.load()
    assert lib.helm_version().decode().startswith("libhelm")


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2405_17696_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.HelmError):
        _lib.load()
