"""The C-ABI library loads and exports every entry point include/*.h declares
(CPU only: no compute calls)."""
import glob
import os
import re

import paper_1803_07772_amd as pa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        names |= set(re.findall(r"ALLOC_API\s+[\w\s\*]+?\b(alloc_\w+)\s*\(", src))
    return names


def test_library_exports_declared_symbols():
    lib = pa.load()
    names = declared_entry_points()
    assert {"alloc_ctx_create", "alloc_ctx_destroy", "alloc_solve", "alloc_params_default",
            "alloc_strerror"} <= names
    for n in names:
        assert hasattr(lib, n), n
    assert set(pa.EXPORTS) <= names


def test_defaults_and_error_strings():
    p = pa.default_params()
    assert p == pa.Params()
    lib = pa.load()
    for code in (0, -22, -12, -5, -27, -2):
        assert lib.alloc_strerror(code)
    assert b"kernel limit" in lib.alloc_strerror(-27)
