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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_arguments_refused_before_any_device_call():
    """create and rhs validate every argument on the host before their first
    HIP call, so the refusals are testable without a GPU (the pointers
    passed here are never dereferenced)."""
    from paper_1908_02464_amd import capi
    lib = ctypes.CDLL(LIB)
    P = ctypes.POINTER(capi.Params)
    vp = ctypes.c_void_p
    lib.weno_l2is_params_default.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.weno_l2is_create.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double, P, vp,
                                                          ctypes.POINTER(vp)]
    lib.weno_l2is_rhs.argtypes = [vp] + [ctypes.c_int] * 3 + [ctypes.c_double, ctypes.c_double, P, vp]
    lib.weno_l2is_strerror.restype = ctypes.c_char_p

    def params(nx, ny, nz, dx=0.1, **kw):
        p = capi.Params()
        assert lib.weno_l2is_params_default(ctypes.byref(p), nx, ny, nz, dx) == capi.OK
        for k, v in kw.items():
            if k == "bc":
                for i, b in enumerate(v):
                    p.bc[i] = b
            else:
                setattr(p, k, v)
        return p

    def create(nx, ny, nz, dx=0.1, gamma=1.4, p=None):
        out = vp(12345)
        p = p if p is not None else params(max(nx, 1), max(ny, 1), max(nz, 1))
        rc = lib.weno_l2is_create(nx, ny, nz, dx, gamma, ctypes.byref(p), None, ctypes.byref(out))
        assert out.value is None  # nothing handed out on failure
        return rc

    assert create(0, 1, 1) == capi.E_SHAPE            # empty grid
    assert create(8, 0, 1) == capi.E_SHAPE
    assert create(8, 1, 4) == capi.E_SHAPE            # nz > 1 with ny == 1
    assert create(65536, 65536, 1) == capi.E_SHAPE     # 2^32 cells: lists address 32 bits
    assert create(4096, 1024, 1024) == capi.E_SHAPE
    assert create(8, 1, 1, dx=-0.1) == capi.E_PARAM
    assert create(8, 1, 1, dx=float("inf")) == capi.E_PARAM
    assert create(8, 1, 1, gamma=1.0) == capi.E_PARAM
    assert create(8, 1, 1, p=params(8, 1, 1, cfl=0.0)) == capi.E_PARAM
    assert create(8, 1, 1, p=params(8, 1, 1, split=7)) == capi.E_PARAM
    assert create(8, 1, 1, p=params(8, 1, 1, bc=[0, 1, 1, 1, 1, 1])) == capi.E_BC   # unpaired periodic
    assert create(2, 1, 1, p=params(2, 1, 1, bc=[2, 2, 1, 1, 1, 1])) == capi.E_BC   # wall needs 3 cells
    p = params(8, 1, 1)
    assert lib.weno_l2is_create(8, 1, 1, 0.1, 1.4, ctypes.byref(p), None, None) == capi.E_NULL
    assert lib.weno_l2is_params_default(ctypes.byref(p), 0, 1, 1, 0.1) == capi.E_SHAPE
    assert lib.weno_l2is_params_default(None, 8, 1, 1, 0.1) == capi.E_NULL
    fake = vp(1 << 40)  # never dereferenced: every call below is refused first
    assert lib.weno_l2is_rhs(None, 8, 1, 1, 0.1, 1.4, ctypes.byref(p), fake) == capi.E_NULL
    assert lib.weno_l2is_rhs(fake, 0, 1, 1, 0.1, 1.4, ctypes.byref(p), vp((1 << 40) + 4096)) == capi.E_SHAPE
    assert lib.weno_l2is_rhs(fake, 8, 1, 1, 0.1, 1.4, ctypes.byref(p), fake) == capi.E_PARAM
    # 3 x 8 doubles = 192 bytes: a dUdt 100 bytes further on still overlaps
    assert lib.weno_l2is_rhs(fake, 8, 1, 1, 0.1, 1.4, ctypes.byref(p), vp((1 << 40) + 100)) == capi.E_PARAM
    for code in (capi.OK, capi.E_NULL, capi.E_SHAPE, capi.E_PARAM, capi.E_BC, capi.E_HIP, capi.E_NOMEM,
                 capi.E_BUDGET, capi.E_SLOT, capi.S_NONPHYSICAL):
        assert lib.weno_l2is_strerror(code)
    # no rhs call has cached a context: releasing touches no device
    assert lib.weno_l2is_rhs_release() == 0
    # the allocation-free rhs refuses, before any device call, grids beyond
    # its static scratch, inflow sides and the refusals of weno_l2is_rhs
    lib.weno_l2is_rhs_noalloc.argtypes = lib.weno_l2is_rhs.argtypes + [vp]
    big = params(4096, 4096, 1)
    assert lib.weno_l2is_rhs_noalloc(fake, 4096, 4096, 1, 0.1, 1.4, ctypes.byref(big), vp((1 << 41)), None) == capi.E_BUDGET
    inflow = params(8, 1, 1, bc=[3, 1, 1, 1, 1, 1])
    assert lib.weno_l2is_rhs_noalloc(fake, 8, 1, 1, 0.1, 1.4, ctypes.byref(inflow), vp((1 << 41)), None) == capi.E_BC
    assert lib.weno_l2is_rhs_noalloc(None, 8, 1, 1, 0.1, 1.4, ctypes.byref(p), fake, None) == capi.E_NULL
    assert lib.weno_l2is_rhs_noalloc(fake, 8, 1, 1, 0.1, 1.4, ctypes.byref(p), fake, None) == capi.E_PARAM
