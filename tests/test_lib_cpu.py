"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "dsweep.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(dsd_[a-z_0-9]+)\s*\(", hdr)))


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2002_05327_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares exactly the header's entry points
    assert set(_lib.EXPORTS) == set(names)


def test_strerror_without_gpu():
    from paper_2002_05327_amd import _lib
    lib = _lib.load()
    assert lib.dsd_strerror(-4).decode().startswith("singular")
    assert lib.dsd_strerror(1).decode().startswith("tolerance")


def test_oracle_is_not_imported_by_the_product():
    pkg = os.path.join(ROOT, "paper_2002_05327_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", txt, re.M), fn
                assert "oracle/" not in txt, fn
