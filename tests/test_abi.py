"""The C-ABI library loads and exports every symbol include/cdsigma.h declares.

No compute call is made (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cdsigma.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cds_[a-z0-9_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    from paper_0912_1459_amd import _lib
    assert _declared() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_0912_1459_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libcdsigma.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    L = _lib.load()
    assert L.cds_version().decode().startswith("cdsigma")


def test_no_cpu_fallback_in_product_path():
    # the package never imports the oracle, and the binding refuses to run without the library
    pkg = os.path.join(ROOT, "paper_0912_1459_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
