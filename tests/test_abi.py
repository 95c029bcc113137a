"""The C-ABI library loads (without a GPU) and exports every entry point that
include/*.h declares; the Python binding names the same entry points.  No
compute call is made here."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1908_02464_amd", "libweno_l2is.so")


def declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"\b(weno_l2is_\w+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_header_declares_entry_points():
    names = declared()
    for n in ("weno_l2is_rhs", "weno_l2is_step", "weno_l2is_create", "weno_l2is_advance",
              "weno_l2is_batch_admit", "weno_l2is_batch_advance"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_declarations():
    src = open(os.path.join(ROOT, "paper_1908_02464_amd", "capi.py")).read()
    bound = set(re.findall(r'"(weno_l2is_\w+)"', src))
    assert declared() <= bound, sorted(declared() - bound)
