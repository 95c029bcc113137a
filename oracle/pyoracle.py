"""ctypes binding of the CPU oracle (test infrastructure only).

The oracle is a plain scalar FP64 C implementation of the L2-norm regularized
incremental-stencil WENO scheme (Zhu & Hu, arXiv 1908.02464).  Only the test
suite, ``__graft_entry__.smoke`` and the CPU-baseline leg of ``bench.py`` may
import this module.  It never serves as a fallback for the GPU library.

Arrays are numpy float64, layout [nvar][nz][ny][nx] (x fastest).
The environment variable ORACLE_L2IS_LIB names another build of the same
sources to load instead (the planted-mistake test loads altered copies of
the oracle this way; the files here are never altered).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(HERE, "liboracle_l2is.so")  # what build() writes
LIB_PATH = os.environ.get("ORACLE_L2IS_LIB") or DEFAULT_LIB  # what lib() loads
SOURCES = ["weno_scalar.c", "charsys.c", "face.c", "solver.c"]

BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE, BC_INFLOW = 0, 1, 2, 3
BC_STATE_WALL, BC_STATE_FRONT = 4, 5
SPLIT_LLF, SPLIT_LF, SPLIT_ROE = 0, 1, 2
HYB_PER_FIELD, HYB_PER_FACE, HYB_WENO_ONLY, HYB_LINEAR_ONLY = 0, 1, 2, 3
W_L2IS, W_IS, W_IS_B01 = 0, 1, 2


def build(verbose: bool = False, src_dir: str = HERE, out: str = DEFAULT_LIB) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction; OpenMP
    over the lines of a sweep, which changes no result bit): the sources in
    src_dir (default: these) into the library out."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-o", out]
    cmd += [os.path.join(src_dir, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


class Params(C.Structure):
    _fields_ = [
        ("cfl", C.c_double),
        ("c_reg", C.c_double),
        ("eps_w", C.c_double),
        ("thr_C", C.c_double),
        ("thr_alpha", C.c_int),
        ("split", C.c_int),
        ("hybrid", C.c_int),
        ("bc", C.c_int * 6),
        ("thr_L", C.c_double * 3),
        ("inflow", C.POINTER(C.c_double)),
        ("weights", C.c_int),
        ("bstate", (C.c_double * 5) * 2),
        ("bgeom", C.c_double * 4),
        ("time", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if LIB_PATH == DEFAULT_LIB and not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_ubyte)
        pp = C.POINTER(Params)
        L.orc_params_default.argtypes = [pp, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_weno_l2is.argtypes = [dp, C.c_double, C.c_double, dp]
        L.orc_weno_l2is.restype = C.c_double
        L.orc_weno.argtypes = [dp, C.c_int, C.c_double, C.c_double, dp]
        L.orc_weno.restype = C.c_double
        L.orc_roe_eigen.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp, dp, dp, dp, dp]
        L.orc_phys_flux.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp, dp]
        L.orc_face_flux.argtypes = [C.c_int, C.c_int, C.c_double, pp, C.c_double,
                                    dp, dp, dp, up, dp]
        grid = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double]
        L.orc_rhs.argtypes = [dp] + grid + [pp, dp]
        L.orc_rhs_at.argtypes = [dp] + grid + [pp, C.c_int,
                                               C.POINTER(C.c_longlong), dp]
        L.orc_face_debug.argtypes = [dp] + grid + [pp, C.c_int, up, dp]
        L.orc_cfl_dt.argtypes = [dp] + grid + [C.c_double, dp]
        L.orc_step.argtypes = [dp] + grid + [pp, C.c_double, dp]
        L.orc_run.argtypes = [dp] + grid + [pp, C.c_double, C.c_int, dp,
                                            C.POINTER(C.c_int)]
        L.orc_threads.argtypes = [C.c_int]
        L.orc_threads.restype = C.c_int
        _lib = L
    return _lib


def threads(n: int = 0) -> int:
    """Set (n > 0) and return the oracle's thread count."""
    return int(lib().orc_threads(int(n)))


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def dims(U: np.ndarray):
    """(nx, ny, nz) of a state array shaped [nvar, nz, ny, nx]."""
    assert U.ndim == 4
    return U.shape[3], U.shape[2], U.shape[1]


def params(nx: int, ny: int, nz: int, dx: float, **kw) -> Params:
    p = Params()
    lib().orc_params_default(C.byref(p), nx, ny, nz, dx)
    for k, v in kw.items():
        if k == "bc":
            for i, b in enumerate(v):
                p.bc[i] = int(b)
        elif k == "bstate":
            for s_, st in enumerate(v):
                for i, x in enumerate(st):
                    p.bstate[s_][i] = float(x)
        elif k == "bgeom":
            for i, b in enumerate(v):
                p.bgeom[i] = float(b)
        elif k == "thr_L":
            for i, b in enumerate(v):
                p.thr_L[i] = float(b)
        elif k == "inflow":
            # conserved ghost state [nvar][ny*nz] of the x- inflow side; the
            # array is kept alive with the structure
            arr = np.ascontiguousarray(v, dtype=np.float64).ravel()
            p._inflow_keep = arr
            p.inflow = arr.ctypes.data_as(C.POINTER(C.c_double))
        else:
            setattr(p, k, v)
    return p


def _check(rc: int, what: str, allow_status: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_status):
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


def weno_l2is(a, lam: float, eps_w: float = 1e-20):
    """Scalar reconstruction; returns (fhat, dict of intermediates)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    dbg = np.zeros(17)
    f = lib().orc_weno_l2is(_dp(a), float(lam), float(eps_w), _dp(dbg))
    return f, {"q": dbg[0:4].copy(), "beta": dbg[4:8].copy(), "tau5": dbg[8],
               "E": dbg[9:13].copy(), "omega": dbg[13:17].copy()}


def weno(a, weights: int, lam: float = 0.0, eps_w: float = 1e-20):
    """Scalar reconstruction with the weights W_*; returns (fhat, dict)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    dbg = np.zeros(17)
    f = lib().orc_weno(_dp(a), int(weights), float(lam), float(eps_w), _dp(dbg))
    return f, {"q": dbg[0:4].copy(), "beta": dbg[4:8].copy(), "tau5": dbg[8],
               "E": dbg[9:13].copy(), "omega": dbg[13:17].copy()}


def roe_eigen(nvar: int, d: int, gamma: float, UL, UR):
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    L = np.zeros((nvar, nvar))
    R = np.zeros((nvar, nvar))
    lam = np.zeros(nvar)
    roe = np.zeros(6)
    _check(lib().orc_roe_eigen(nvar, d, gamma, _dp(UL), _dp(UR), _dp(L), _dp(R),
                               _dp(lam), _dp(roe)), "roe_eigen")
    return L, R, lam, roe


def phys_flux(nvar: int, d: int, gamma: float, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    F = np.zeros(nvar)
    prim = np.zeros(7)
    _check(lib().orc_phys_flux(nvar, d, gamma, _dp(U), _dp(F), _dp(prim)), "phys_flux")
    return F, prim


def face_flux(nvar: int, d: int, gamma: float, p: Params, eps_thr: float, U6,
              alpha_lf=None):
    U6 = np.ascontiguousarray(U6, dtype=np.float64).reshape(6, nvar)
    a = np.zeros(nvar) if alpha_lf is None else np.ascontiguousarray(alpha_lf, dtype=np.float64)
    F = np.zeros(nvar)
    fl = np.zeros(nvar, dtype=np.uint8)
    sg = np.zeros(nvar)
    _check(lib().orc_face_flux(nvar, d, gamma, C.byref(p), eps_thr, _dp(a), _dp(U6),
                               _dp(F), fl.ctypes.data_as(C.POINTER(C.c_ubyte)), _dp(sg)),
           "face_flux")
    return F, fl, sg


def rhs(U: np.ndarray, dx: float, gamma: float, p: Params) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    nx, ny, nz = dims(U)
    out = np.zeros_like(U)
    _check(lib().orc_rhs(_dp(U), nx, ny, nz, dx, gamma, C.byref(p), _dp(out)), "rhs")
    return out


def rhs_at(U: np.ndarray, dx: float, gamma: float, p: Params, cells) -> np.ndarray:
    """dU/dt at flat cell indices x + nx*(y + ny*z); returns [nvar, ncells]."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    nx, ny, nz = dims(U)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((U.shape[0], cells.size))
    _check(lib().orc_rhs_at(_dp(U), nx, ny, nz, dx, gamma, C.byref(p), int(cells.size),
                            cells.ctypes.data_as(C.POINTER(C.c_longlong)), _dp(out)),
           "rhs_at")
    return out


def face_debug(U: np.ndarray, dx: float, gamma: float, p: Params, d: int):
    U = np.ascontiguousarray(U, dtype=np.float64)
    nx, ny, nz = dims(U)
    shp = [U.shape[0], nz, ny, nx]
    shp[3 - d] += 1
    fl = np.zeros(shp, dtype=np.uint8)
    sg = np.zeros(shp)
    _check(lib().orc_face_debug(_dp(U), nx, ny, nz, dx, gamma, C.byref(p), d,
                                fl.ctypes.data_as(C.POINTER(C.c_ubyte)), _dp(sg)),
           "face_debug")
    return fl, sg


def cfl_dt(U: np.ndarray, dx: float, gamma: float, cfl: float = 0.5):
    U = np.ascontiguousarray(U, dtype=np.float64)
    nx, ny, nz = dims(U)
    dt = C.c_double(0.0)
    st = _check(lib().orc_cfl_dt(_dp(U), nx, ny, nz, dx, gamma, cfl, C.byref(dt)),
                "cfl_dt", allow_status=True)
    return dt.value, st


def step(U: np.ndarray, dx: float, gamma: float, p: Params, dt: float = -1.0):
    """One SSP-RK3 step in place; returns (dt_used, status)."""
    assert U.dtype == np.float64 and U.flags.c_contiguous
    nx, ny, nz = dims(U)
    dtu = C.c_double(0.0)
    st = _check(lib().orc_step(_dp(U), nx, ny, nz, dx, gamma, C.byref(p), dt,
                               C.byref(dtu)), "step", allow_status=True)
    return dtu.value, st


def run(U: np.ndarray, dx: float, gamma: float, p: Params, t_end: float,
        max_steps: int = 1 << 30):
    """Advance in place to t_end; returns (t, steps, status)."""
    assert U.dtype == np.float64 and U.flags.c_contiguous
    nx, ny, nz = dims(U)
    t = C.c_double(0.0)
    n = C.c_int(0)
    st = _check(lib().orc_run(_dp(U), nx, ny, nz, dx, gamma, C.byref(p), t_end,
                              max_steps, C.byref(t), C.byref(n)), "run", allow_status=True)
    return t.value, n.value, st
