"""The C-ABI library loads and exports every function include/tigas.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

from paper_2605_08699_amd import tigas

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tigas.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tigas_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert sorted(tigas.EXPORTS) == _declared()


@pytest.mark.skipif(not os.path.exists(tigas.LIB_PATH), reason="libtigas.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(tigas.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(tigas, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(tigas, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        tigas.lib()
