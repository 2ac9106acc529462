"""Host-side checks of the C ABI (no GPU needed): the built library loads and
exports every entry point declared in include/mlmc.h, and the Python
binding's record layouts match the header."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mlmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlmc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1907_10271_amd import _lib
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 13
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib.EXPORTS)


def test_record_layouts_match_header():
    from paper_1907_10271_amd import _lib
    assert C.sizeof(_lib.Request) == 16
    assert C.sizeof(_lib.Info) == 32
    assert C.sizeof(_lib.LevelAcc) == 3 * 8 + 9 * 8


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1907_10271_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "oracle/" not in src.replace("oracle/ ", ""), f


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1907_10271_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="HIP library missing"):
        _lib.load()
