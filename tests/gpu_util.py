"""Helpers shared by the GPU tests (no scheme arithmetic here)."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def z20(a: np.ndarray, b: np.ndarray) -> float:
    """max over cells and variables of |a-b| / max(|b|, max_grid |b_c|)."""
    worst = 0.0
    for c in range(b.shape[0]):
        bc = b[c]
        s = np.maximum(np.abs(bc), np.abs(bc).max())
        s = np.where(s > 0, s, 1.0)
        worst = max(worst, float((np.abs(a[c] - bc) / s).max()))
    return worst


def to_dev(U: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(U)).cuda()


def to_host(t) -> np.ndarray:
    return t.cpu().numpy()


def params_pair(orc, capi, shape, dx, **kw):
    """The same settings for the oracle and the library."""
    nx, ny, nz = shape
    po = orc.params(nx, ny, nz, dx, **{("eps_w" if k == "eps_weno" else k): v for k, v in kw.items()})
    pg = capi.params_default(nx, ny, nz, dx, **kw)
    return po, pg


def rhs_err(a: np.ndarray, b: np.ndarray, U: np.ndarray, dt: float) -> float:
    """dU/dt difference in units of the state after one CFL step:
    max over variables of max|a_c - b_c| * dt / max|U_c|.  (dU/dt itself may
    be ~0 for a component by cancellation between directions, e.g. density
    on a solenoidal field, so it is not a usable scale.)"""
    worst = 0.0
    for c in range(b.shape[0]):
        s = float(np.abs(U[c]).max())
        s = s if s > 0 else 1.0
        worst = max(worst, float(np.abs(a[c] - b[c]).max()) * dt / s)
    return worst
