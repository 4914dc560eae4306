"""The C-ABI library loads and exports every entry point declared in include/nbgs.h (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(nbgs_[a-z_0-9]+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for want in ("nbgs_scene_create", "nbgs_detect", "nbgs_solve", "nbgs_integrate", "nbgs_step"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_1501_05810_amd as nb

    L = ctypes.CDLL(nb.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert sorted(n for n, _, _ in nb._SIGNATURES) == _declared()
    assert nb.nbgs_abi_version() == 1


def test_binding_has_no_cpu_fallback(tmp_path, monkeypatch):
    import paper_1501_05810_amd as nb

    monkeypatch.setattr(nb, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(nb, "_lib", None)
    with pytest.raises(ImportError):
        nb.lib()


def test_oracle_is_not_imported_by_the_product():
    pkg = os.path.join(ROOT, "paper_1501_05810_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "nbgs_ref" not in txt, f
