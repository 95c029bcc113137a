"""The allocation-free right-hand side (weno_l2is_rhs_noalloc) against the
allocating one (weno_l2is_rhs), through the C ABI: the same bits, on a
stream of the caller's, for 1D, 2D and 3D grids and scheme variants, twice
in a row with the second grid smaller (the shared static scratch keeps the
first call's contents), with no change of the device's free memory."""
import ctypes as C

import numpy as np
import pytest

from paper_1908_02464_amd import workloads as w
from gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu
G = 1.4


@pytest.fixture(scope="module")
def capi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1908_02464_amd import capi as c
    c.lib()
    return c


def _turb(nx, ny, nz, seed):
    U, dx = w.turbulence_3d(nx, seed, ny=ny, nz=nz)
    U = np.ascontiguousarray(U.copy())
    U[0, :, :, : nx // 2] *= 2.0  # a contact: nonlinear faces
    U[4, :, :, : nx // 2] *= 2.0
    return U, dx


def _pairs():
    """(first, second) cases: the second grid smaller than the first."""
    q1 = w.four_quadrant_2d(520, 300, 31)
    q2 = w.four_quadrant_2d(67, 45, 11)
    s1 = w.shu_osher(1600)
    s2 = w.sod(200)
    t1 = _turb(40, 36, 30, 5)
    t2 = _turb(20, 18, 17, 6)
    return [
        ("1d", (s1[0], s1[1], [1] * 6, {}), (s2[0], s2[1], [1] * 6, {})),
        ("2d", (q1[0], q1[1], [1] * 6, {}), (q2[0], q2[1], [0, 0, 2, 2, 1, 1], {"hybrid": 1})),
        # global LF: the speed reduction's slots live in the static scratch
        ("2d_lf", (q1[0], q1[1], [1] * 6, {"split": 1}), (q2[0], q2[1], [1] * 6, {"split": 1})),
        ("3d", (t1[0], t1[1], [0] * 6, {}), (t2[0], t2[1], [0] * 6, {"split": 2})),
        ("3d_weno_only", (t1[0], t1[1], [0] * 6, {"hybrid": 2}), (t2[0], t2[1], [1, 1, 2, 2, 0, 0], {"split": 1})),
        ("2d_to_1d", (q1[0], q1[1], [1] * 6, {"weights": 2}), (s2[0], s2[1], [2, 2, 1, 1, 1, 1], {"hybrid": 2})),
    ]


def shape_of(U):
    return U.shape[3], U.shape[2], U.shape[1]


@pytest.mark.parametrize("name", [p[0] for p in _pairs()])
def test_noalloc_rhs_equals_rhs(capi, name):
    import torch
    pair = [p for p in _pairs() if p[0] == name][0]
    stream = torch.cuda.Stream()
    free = []
    for k, (U, dx, bc, kw) in enumerate(pair[1:]):
        shape = shape_of(U)
        say(f"[noalloc] {name} call {k + 1}: shape={shape} kw={kw}")
        p = capi.params_default(*shape, dx, bc=bc, **kw)
        Ud = to_dev(U)
        ref = torch.full_like(Ud, float("nan"))
        capi.rhs(Ud, *shape, dx, G, p, ref)
        got = torch.full_like(Ud, float("nan"))
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
        capi.rhs_noalloc(Ud, *shape, dx, G, p, got, stream=stream)
        stream.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
        a, b = to_host(got), to_host(ref)
        assert np.all(np.isfinite(a))
        d = float(np.abs(a - b).max())
        say(f"    max |noalloc - rhs| = {d:.3e}")
        assert np.array_equal(a, b)
    # Nothing allocated on the device: both calls once more, with free
    # device memory read around them.  (The first launch of a build that
    # keeps spilled registers in private memory makes the HIP runtime
    # reserve that memory for the queue; the calls above have done so.)
    args = []
    for U, dx, bc, kw in pair[1:]:
        shape = shape_of(U)
        Ud = to_dev(U)
        args.append((Ud, shape, dx, capi.params_default(*shape, dx, bc=bc, **kw), torch.empty_like(Ud)))
    torch.cuda.synchronize()
    before = torch.cuda.mem_get_info()[0]
    for Ud, shape, dx, p, got in args:
        capi.rhs_noalloc(Ud, *shape, dx, G, p, got, stream=stream)
    stream.synchronize()
    after = torch.cuda.mem_get_info()[0]
    say(f"    free device memory before / after the repeated calls: {before} / {after}")
    assert after == before, (before, after, free)


def test_noalloc_rhs_refusals(capi):
    """Grids beyond the static scratch and inflow sides are refused before
    any device work; null pointers as weno_l2is_rhs."""
    L = capi.lib()
    # addresses far apart that are never dereferenced: every call below is
    # refused on the host
    u, o = C.c_void_p(1 << 40), C.c_void_p(1 << 42)
    big = (4096, 4096, 1)  # 16.8M cells: 134 MB of list
    p = capi.params_default(*big, 0.1)
    assert L.weno_l2is_rhs_noalloc(u, *big, 0.1, G, C.byref(p), o, None) == capi.E_BUDGET
    p = capi.params_default(8, 1, 1, 0.1, bc=[3, 1, 1, 1, 1, 1])
    assert L.weno_l2is_rhs_noalloc(u, 8, 1, 1, 0.1, G, C.byref(p), o, None) == capi.E_BC
    p = capi.params_default(8, 1, 1, 0.1)
    assert L.weno_l2is_rhs_noalloc(None, 8, 1, 1, 0.1, G, C.byref(p), o, None) == capi.E_NULL
