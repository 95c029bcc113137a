"""Thin ctypes binding of libweno_l2is.so (argument marshalling only).

Every function keeps the C name without the ``weno_l2is_`` prefix and takes
torch CUDA float64 tensors where the C call takes device pointers.  All work
runs in the library's HIP kernels; there is no host fallback: a missing or
unloadable library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # loads the HIP runtime that the library then shares

from . import build as _build

LIB_PATH = _build.LIB

OK, E_NULL, E_SHAPE, E_PARAM, E_BC, E_HIP, E_NOMEM, E_BUDGET, E_SLOT = 0, -1, -2, -3, -4, -5, -6, -7, -8
S_NONPHYSICAL = 1
BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE, BC_INFLOW, BC_STATE_WALL, BC_STATE_FRONT = 0, 1, 2, 3, 4, 5
SPLIT_LLF, SPLIT_LF, SPLIT_ROE = 0, 1, 2
HYB_PER_FIELD, HYB_PER_FACE, HYB_WENO_ONLY, HYB_LINEAR_ONLY = 0, 1, 2, 3
PATH_AUTO, PATH_SWEEPS, PATH_FUSED, PATH_FUSED_CELLS = 0, 1, 2, 3


class WenoL2ISError(RuntimeError):
    pass


class Params(C.Structure):
    _fields_ = [
        ("cfl", C.c_double),
        ("c_reg", C.c_double),
        ("eps_weno", C.c_double),
        ("thr_C", C.c_double),
        ("thr_alpha", C.c_int),
        ("split", C.c_int),
        ("hybrid", C.c_int),
        ("bc", C.c_int * 6),
        ("thr_L", C.c_double * 3),
        ("weights", C.c_int),
        ("bstate", (C.c_double * 5) * 2),
        ("bgeom", C.c_double * 4),
    ]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        _build.build()
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.c_double, C.c_int
    pp = C.POINTER(Params)
    sig = {
        "weno_l2is_params_default": (ip, [pp, ip, ip, ip, dp]),
        "weno_l2is_create": (ip, [ip, ip, ip, dp, dp, pp, vp, C.POINTER(vp)]),
        "weno_l2is_rhs": (ip, [vp, ip, ip, ip, dp, dp, pp, vp]),
        "weno_l2is_rhs_ctx": (ip, [vp, vp, vp]),
        "weno_l2is_rhs_release": (ip, []),
        "weno_l2is_rhs_noalloc": (ip, [vp, ip, ip, ip, dp, dp, pp, vp, vp]),
        "weno_l2is_step": (ip, [vp, vp, dp]),
        "weno_l2is_advance": (ip, [vp, vp, ip, dp]),
        "weno_l2is_set_time": (ip, [vp, dp]),
        "weno_l2is_set_inflow": (ip, [vp, vp]),
        "weno_l2is_cfl_dt": (ip, [vp, vp, C.POINTER(dp)]),
        "weno_l2is_time": (ip, [vp, C.POINTER(dp), C.POINTER(dp), C.POINTER(C.c_uint)]),
        "weno_l2is_face_debug": (ip, [vp, vp, ip, vp, vp]),
        "weno_l2is_status": (ip, [vp, C.POINTER(C.c_uint), ip]),
        "weno_l2is_tune": (ip, [vp, ip, ip, ip]),
        "weno_l2is_timing_enable": (ip, [vp, ip]),
        "weno_l2is_timing_read": (ip, [vp, ip, C.c_char_p, C.POINTER(dp), C.POINTER(C.c_longlong),
                                       C.POINTER(ip)]),
        "weno_l2is_destroy": (None, [vp]),
        "weno_l2is_batch_create": (ip, [C.c_size_t, ip, vp, C.POINTER(vp)]),
        "weno_l2is_batch_admit": (ip, [vp, ip, ip, ip, dp, dp, pp, vp, ip, dp,
                                       C.POINTER(ip), C.POINTER(C.c_size_t)]),
        "weno_l2is_batch_advance": (ip, [vp, ip]),
        "weno_l2is_batch_poll": (ip, [vp, C.POINTER(ip), ip, C.POINTER(ip)]),
        "weno_l2is_batch_fetch": (ip, [vp, ip, vp, ip, C.POINTER(dp), C.POINTER(C.c_uint),
                                       C.POINTER(C.c_uint)]),
        "weno_l2is_batch_usage": (ip, [vp, C.POINTER(C.c_size_t), C.POINTER(ip)]),
        "weno_l2is_batch_tune": (ip, [vp, ip, ip]),
        "weno_l2is_batch_destroy": (None, [vp]),
        "weno_l2is_strerror": (C.c_char_p, [ip]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def strerror(code: int) -> str:
    return lib().weno_l2is_strerror(int(code)).decode()


def _chk(rc: int, what: str, allow_status: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_status):
        raise WenoL2ISError(f"weno_l2is_{what}: {strerror(rc)} ({rc})")
    return rc


def _ptr(t: torch.Tensor, numel: int, dtype=torch.float64) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise WenoL2ISError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise WenoL2ISError(f"expected contiguous {dtype} with {numel} elements")
    return t.data_ptr()


def grid_dims(nx: int, ny: int, nz: int):
    dim = 3 if nz > 1 else (2 if ny > 1 else 1)
    return dim, dim + 2, nx * ny * nz


def params_default(nx: int, ny: int, nz: int, dx: float, **kw) -> Params:
    p = Params()
    _chk(lib().weno_l2is_params_default(C.byref(p), nx, ny, nz, dx), "params_default")
    for k, v in kw.items():
        if k in ("bc", "thr_L", "bgeom"):
            arr = getattr(p, k)
            for i, b in enumerate(v):
                arr[i] = b
        elif k == "bstate":
            for s, st in enumerate(v):
                for i, x in enumerate(st):
                    p.bstate[s][i] = float(x)
        else:
            setattr(p, k, v)
    return p


def rhs(U: torch.Tensor, nx: int, ny: int, nz: int, dx: float, gamma: float, params: Params,
        dUdt: torch.Tensor) -> None:
    """Stateless right-hand side on the null stream (weno_l2is_rhs)."""
    _, nvar, ncell = grid_dims(nx, ny, nz)
    _chk(lib().weno_l2is_rhs(_ptr(U, nvar * ncell), nx, ny, nz, dx, gamma, C.byref(params),
                             _ptr(dUdt, nvar * ncell)), "rhs")


def rhs_noalloc(U: torch.Tensor, nx: int, ny: int, nz: int, dx: float, gamma: float,
                params: Params, dUdt: torch.Tensor, stream=None) -> None:
    """weno_l2is_rhs without device allocation (static scratch), on `stream`
    (a torch stream; None: the current one)."""
    _, nvar, ncell = grid_dims(nx, ny, nz)
    s = stream if stream is not None else torch.cuda.current_stream()
    _chk(lib().weno_l2is_rhs_noalloc(_ptr(U, nvar * ncell), nx, ny, nz, dx, gamma, C.byref(params),
                                     _ptr(dUdt, nvar * ncell), C.c_void_p(s.cuda_stream)), "rhs_noalloc")


def rhs_release() -> int:
    """Free the contexts cached by the stateless rhs (weno_l2is_rhs_release);
    returns how many were released."""
    n = lib().weno_l2is_rhs_release()
    _chk(min(n, 0), "rhs_release")
    return n


class Context:
    """Owns a weno_l2is_ctx (one grid, its stream, scratch and device clock)."""

    def __init__(self, nx: int, ny: int, nz: int, dx: float, gamma: float = 1.4,
                 params: Params | None = None, stream: torch.cuda.Stream | None = None):
        self.shape = (nx, ny, nz)
        self.dim, self.nvar, self.ncell = grid_dims(nx, ny, nz)
        self.dx, self.gamma = dx, gamma
        self.params = params if params is not None else params_default(nx, ny, nz, dx)
        st = stream if stream is not None else torch.cuda.current_stream()
        self.stream = st
        h = C.c_void_p()
        _chk(lib().weno_l2is_create(nx, ny, nz, dx, gamma, C.byref(self.params),
                                    C.c_void_p(st.cuda_stream), C.byref(h)), "create")
        self.h = h

    def _u(self, t):
        return _ptr(t, self.nvar * self.ncell)

    def rhs(self, U, dUdt):
        _chk(lib().weno_l2is_rhs_ctx(self.h, self._u(U), self._u(dUdt)), "rhs_ctx")

    def step(self, U, dt: float = -1.0):
        _chk(lib().weno_l2is_step(self.h, self._u(U), float(dt)), "step")

    def advance(self, U, n_steps: int, t_end: float):
        _chk(lib().weno_l2is_advance(self.h, self._u(U), int(n_steps), float(t_end)), "advance")

    def set_inflow(self, state):
        """Ghost state of the x- inflow side: conserved [nvar][ny*nz] (device)."""
        _chk(lib().weno_l2is_set_inflow(self.h, _ptr(state, self.nvar * self.shape[1] * self.shape[2])),
             "set_inflow")

    def set_time(self, t: float):
        _chk(lib().weno_l2is_set_time(self.h, float(t)), "set_time")

    def cfl_dt(self, U):
        dt = C.c_double(0.0)
        st = _chk(lib().weno_l2is_cfl_dt(self.h, self._u(U), C.byref(dt)), "cfl_dt", True)
        return dt.value, st

    def time(self):
        """(device clock, dt of the latest step)."""
        return self.clock()[:2]

    def clock(self):
        """(device clock, dt of the latest step, clock steps taken)."""
        t, dt, n = C.c_double(0.0), C.c_double(0.0), C.c_uint(0)
        _chk(lib().weno_l2is_time(self.h, C.byref(t), C.byref(dt), C.byref(n)), "time")
        return t.value, dt.value, n.value

    def face_debug(self, U, d: int, flags, sigma):
        nf = self.ncell // self.shape[d] * (self.shape[d] + 1)
        _chk(lib().weno_l2is_face_debug(self.h, self._u(U), d,
                                        _ptr(flags, self.nvar * nf, torch.uint8),
                                        _ptr(sigma, self.nvar * nf)), "face_debug")

    def status(self, clear: bool = False) -> int:
        bits = C.c_uint(0)
        _chk(lib().weno_l2is_status(self.h, C.byref(bits), int(clear)), "status", True)
        return bits.value

    def tune(self, path: int = 0, zchunk: int = 0, waves_per_simd: int = 0):
        _chk(lib().weno_l2is_tune(self.h, int(path), int(zchunk), int(waves_per_simd)), "tune")

    def timing(self, enable: bool):
        _chk(lib().weno_l2is_timing_enable(self.h, int(enable)), "timing_enable")

    def timing_read(self, cap: int = 32):
        """{kernel name: (total_ms, launches)} of the launches since enable."""
        names = C.create_string_buffer(64 * cap)
        tot = (C.c_double * cap)()
        cnt = (C.c_longlong * cap)()
        n = C.c_int(0)
        _chk(lib().weno_l2is_timing_read(self.h, cap, names, tot, cnt, C.byref(n)), "timing_read")
        out = {}
        for k in range(n.value):
            nm = names.raw[64 * k: 64 * k + 64].split(b"\0", 1)[0].decode()
            out[nm] = (tot[k], cnt[k])
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().weno_l2is_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owns a weno_l2is_batch engine (batched / served runs, 1D and 2D)."""

    def __init__(self, budget_bytes: int, max_slots: int = 1024,
                 stream: torch.cuda.Stream | None = None):
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        _chk(lib().weno_l2is_batch_create(int(budget_bytes), int(max_slots),
                                          C.c_void_p(self.stream.cuda_stream), C.byref(h)),
             "batch_create")
        self.h = h
        self.meta = {}

    def admit(self, U0, nx: int, ny: int, nz: int, dx: float, t_end: float,
              gamma: float = 1.4, params: Params | None = None):
        """Admit a run; U0 is a host numpy float64 array or a CUDA tensor.
        Returns the slot, or None when the budget or the slot table is full."""
        import numpy as np
        p = params if params is not None else params_default(nx, ny, nz, dx)
        slot, nbytes = C.c_int(-1), C.c_size_t(0)
        if isinstance(U0, torch.Tensor):
            ptr, host = _ptr(U0, U0.numel()), 0
        else:
            U0 = np.ascontiguousarray(U0, dtype=np.float64)
            ptr, host = U0.ctypes.data, 1
        rc = lib().weno_l2is_batch_admit(self.h, nx, ny, nz, dx, gamma, C.byref(p), C.c_void_p(ptr),
                                         host, float(t_end), C.byref(slot), C.byref(nbytes))
        if rc == E_BUDGET:
            return None
        _chk(rc, "batch_admit")
        self.meta[slot.value] = (nx, ny, nz)
        return slot.value

    def advance(self, n_steps: int = 1):
        _chk(lib().weno_l2is_batch_advance(self.h, int(n_steps)), "batch_advance")

    def poll(self, cap: int = 4096):
        arr = (C.c_int * cap)()
        n = C.c_int(0)
        _chk(lib().weno_l2is_batch_poll(self.h, arr, cap, C.byref(n)), "batch_poll")
        return [arr[i] for i in range(n.value)]

    def fetch(self, slot: int, with_steps: bool = False):
        """Copy the run's state to a host array, free the slot.
        Returns (U, t, status), or (U, t, status, steps) with with_steps."""
        import numpy as np
        if slot not in self.meta:
            raise WenoL2ISError(f"weno_l2is_batch_fetch: slot {slot} holds no run")
        nx, ny, nz = self.meta.pop(slot)
        dim, nvar, ncell = grid_dims(nx, ny, nz)
        U = np.empty((nvar, nz, ny, nx))
        t, st, n = C.c_double(0.0), C.c_uint(0), C.c_uint(0)
        _chk(lib().weno_l2is_batch_fetch(self.h, int(slot), C.c_void_p(U.ctypes.data), 1,
                                         C.byref(t), C.byref(st), C.byref(n)), "batch_fetch")
        return (U, t.value, st.value, n.value) if with_steps else (U, t.value, st.value)

    def tune(self, rows: int = 0, blocks: int = 0):
        """Rows per work item of the 2D runs and persistent grid size of the
        batched stage kernels; 0 keeps the current value."""
        _chk(lib().weno_l2is_batch_tune(self.h, int(rows), int(blocks)), "batch_tune")

    def usage(self):
        used, act = C.c_size_t(0), C.c_int(0)
        _chk(lib().weno_l2is_batch_usage(self.h, C.byref(used), C.byref(act)), "batch_usage")
        return used.value, act.value

    def close(self):
        if getattr(self, "h", None):
            lib().weno_l2is_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
