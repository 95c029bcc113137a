"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds initial states (and request streams); it contains
none of the scheme's arithmetic.  The same float64 bytes feed the GPU library
and the CPU oracle.  Every state is a numpy array [nvar][nz][ny][nx] of
conserved variables (rho, rho*u, [rho*v, [rho*w]], E) with
E = p/(gamma-1) + rho|u|^2/2 (the ideal-gas closure of the Euler equations).
Grids are cell centred: x_i = x0 + (i + 1/2) dx; a point exactly on an
interface takes the right-hand state.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4


def conserved(rho, vel, p, gamma=GAMMA):
    """Stack primitive fields into conserved variables [nvar, ...]."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape) for v in vel]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    ke = 0.5 * rho * sum(v * v for v in vel)
    comps = [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke]
    return np.ascontiguousarray(np.stack(comps))


def centres(n, x0, x1):
    dx = (x1 - x0) / n
    return x0 + (np.arange(n) + 0.5) * dx, dx


# ----------------------------------------------------------------------------- 1D
def riemann_1d(n, left, right, x_int=0.5, x0=0.0, x1=1.0, gamma=GAMMA):
    """Two-state problem; left/right = (rho, u, p).  Returns (U[3,1,1,n], dx)."""
    x, dx = centres(n, x0, x1)
    L = x < x_int
    rho = np.where(L, left[0], right[0])
    u = np.where(L, left[1], right[1])
    p = np.where(L, left[2], right[2])
    return conserved(rho, [u], p, gamma).reshape(3, 1, 1, n), dx


SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
LAX = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.5710))
PROBLEM_123 = ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4))


def sod(n=200):
    """Sod shock tube on [0,1], interface 0.5 (Sec. 4.2)."""
    return riemann_1d(n, *SOD)


def sound_packet(n=128, seed=0, k0=12.0, eps=1e-3, gamma=GAMMA):
    """Broadband acoustic packet on [0,1], periodic (Sec. 4.1, Eq.(36)-(37)):
    p = p0 (1 + eps sum_{k=0}^{n/2} sqrt(E_p(k)) sin(2 pi k (x + phi_k))) with
    E_p(k) = (k/k0)^4 exp(-2 (k/k0)^2) and phases phi_k uniform in [0,1),
    isentropic rho = rho0 (p/p0)^(1/gamma), and the velocity of a
    right-running simple wave u = u0 + 2 (c - c0)/(gamma - 1) (the printed
    velocity is garbled; this is the reading).  rho0 = 1, p0 = 1/gamma
    (c0 = 1), u0 = 0, so one period is t = 1."""
    x, dx = centres(n, 0.0, 1.0)
    rng = np.random.default_rng(seed)
    k = np.arange(n // 2 + 1, dtype=np.float64)
    phi = rng.random(k.size)
    amp = np.sqrt((k / k0) ** 4 * np.exp(-2.0 * (k / k0) ** 2))
    p0, rho0 = 1.0 / gamma, 1.0
    p = p0 * (1.0 + eps * (amp[:, None] * np.sin(2.0 * np.pi * k[:, None] * (x[None, :] + phi[:, None]))).sum(0))
    rho = rho0 * (p / p0) ** (1.0 / gamma)
    c = np.sqrt(gamma * p / rho)
    u = 2.0 * (c - 1.0) / (gamma - 1.0)
    return conserved(rho, [u], p, gamma).reshape(3, 1, 1, n), dx


def blast_waves(n=400, gamma=GAMMA):
    """Two interacting blast waves on [0,1] (Sec. 4.3): rho = 1, u = 0 and
    p = 1000 / 0.01 / 100 on [0, 0.1) / [0.1, 0.9) / [0.9, 1]; reflective
    walls at both ends, Roe-speed splitting, t_end = 0.038."""
    x, dx = centres(n, 0.0, 1.0)
    p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0))
    return conserved(np.ones(n), [np.zeros(n)], p, gamma).reshape(3, 1, 1, n), dx


JET_GAMMA = 5.0 / 3.0


def mach2000_jet(nx=640, ny=160, gamma=JET_GAMMA):
    """Mach 2000 jet (Sec. 4.7) on [0,1] x [0,0.25]: ambient gas
    (rho, u, v, p) = (0.5, 0, 0, 0.4127) everywhere; the left side is an
    inflow whose ghosts hold the jet (5, 800, 0, 0.4127) for y < 0.05 and
    the ambient state above; reflective bottom, outflow right and top;
    gamma = 5/3, CFL 0.25, t_end = 0.001.  Returns (U0, dx, inflow), inflow
    the conserved ghost state [4][ny]."""
    x, dx = centres(nx, 0.0, 1.0)
    y, _ = centres(ny, 0.0, 0.25)
    rho = np.full((ny, nx), 0.5)
    zero = np.zeros((ny, nx))
    U0 = conserved(rho, [zero, zero], np.full((ny, nx), 0.4127), gamma).reshape(4, 1, ny, nx)
    jet = y < 0.05
    inflow = conserved(np.where(jet, 5.0, 0.5), [np.where(jet, 800.0, 0.0), np.zeros(ny)],
                       np.full(ny, 0.4127), gamma)
    return U0, dx, np.ascontiguousarray(inflow.reshape(4, ny))


DMR_PRE = (1.4, 0.0, 0.0, 1.0)
DMR_POST = (8.0, 7.145, -4.125, 116.8333)
DMR_X0, DMR_SLOPE = 0.1667, 1.732


def double_mach(nx=512, ny=128, gamma=GAMMA):
    """Double Mach reflection (Sec. 4.5) on [0,4] x [0,1] (nx = 4 ny): the
    Mach 10 shock y = 1.732 (x - 0.1667) with the pre-shock gas (1.4, 0, 0,
    1) below-right of it and (8, 7.145, -4.125, 116.8333) above-left (the
    printed states; a cell takes the pre-shock state when its centre is on
    or below the line).  Returns (U0, dx, params): the boundary settings of
    the run, keyword arguments of the oracle's and the library's parameter
    constructors: post-shock inflow on the left; outflow on the right; the
    bottom a wall from x = 0.1667 on and the post-shock state left of it;
    the top the exact position of the moving shock, x = 0.1667 + (y + 20 t)
    / 1.732 (the shock moves at 10 normal to itself into gas with sound speed
    1), post-shock left of it and pre-shock right of it; global LF splitting
    (the paper's splitting for its 2D cases)."""
    assert nx == 4 * ny
    x, dx = centres(nx, 0.0, 4.0)
    y, _ = centres(ny, 0.0, 1.0)
    X, Y = np.meshgrid(x, y)
    pre = Y <= DMR_SLOPE * (X - DMR_X0)
    prim = [np.where(pre, a, b) for a, b in zip(DMR_PRE, DMR_POST)]
    U0 = conserved(prim[0], [prim[1], prim[2]], prim[3], gamma).reshape(4, 1, ny, nx)
    post = conserved(np.array(DMR_POST[0]), [np.array(DMR_POST[1]), np.array(DMR_POST[2])],
                     np.array(DMR_POST[3]), gamma).ravel()
    pre_s = conserved(np.array(DMR_PRE[0]), [np.array(DMR_PRE[1]), np.array(DMR_PRE[2])],
                      np.array(DMR_PRE[3]), gamma).ravel()
    inflow = np.ascontiguousarray(np.repeat(post.reshape(4, 1), ny, axis=1))
    params = {"bc": [3, 1, 4, 5, 1, 1], "split": 1,
              "bstate": [list(post) + [0.0], list(pre_s) + [0.0]],
              # wall from x = 0.1667; front x0, dx/dy, dx/dt
              "bgeom": [DMR_X0, DMR_X0, 1.0 / DMR_SLOPE, 20.0 / DMR_SLOPE]}
    return np.ascontiguousarray(U0), dx, params, inflow


def shu_osher(n=1600, gamma=GAMMA):
    """Mach-3 shock / entropy wave on [-5,5]: shocked state for x < -4."""
    x, dx = centres(n, -5.0, 5.0)
    L = x < -4.0
    rho = np.where(L, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
    u = np.where(L, 2.629369, 0.0)
    p = np.where(L, 10.33333, 1.0)
    return conserved(rho, [u], p, gamma).reshape(3, 1, 1, n), dx


def smooth_advection(n, gamma=GAMMA):
    """rho = 1 + 0.2 sin(pi x), u = 1, p = 1 on [-1,1], periodic."""
    x, dx = centres(n, -1.0, 1.0)
    rho = 1.0 + 0.2 * np.sin(np.pi * x)
    return conserved(rho, [np.ones(n)], np.ones(n), gamma).reshape(3, 1, 1, n), dx


def smooth_advection_exact(n, t, gamma=GAMMA):
    x, dx = centres(n, -1.0, 1.0)
    rho = 1.0 + 0.2 * np.sin(np.pi * (x - t))
    return conserved(rho, [np.ones(n)], np.ones(n), gamma).reshape(3, 1, 1, n)


# -------------------------------------------------------------- random states
def _no_vacuum(a, b, gamma):
    """Pressure-positivity condition of the exact Riemann solution."""
    ca = math.sqrt(gamma * a[3] / a[0])
    cb = math.sqrt(gamma * b[3] / b[0])
    return (b[1] - a[1]) < 2.0 * (ca + cb) / (gamma - 1.0)


def random_quadrants(rng, gamma=GAMMA):
    """Four (rho, u, v, p) states, rho in [0.1,1.5], u,v in [-1,1],
    p in [0.03,1.5]; redrawn until no interface generates vacuum and at least
    one interface is compressive (a shock/contact mix)."""
    while True:
        q = np.column_stack([rng.uniform(0.1, 1.5, 4), rng.uniform(-1, 1, 4),
                             rng.uniform(-1, 1, 4), rng.uniform(0.03, 1.5, 4)])
        # quadrants: 0 = (x>.5,y>.5), 1 = (x<.5,y>.5), 2 = (x<.5,y<.5), 3 = (x>.5,y<.5)
        pairs_x = [(1, 0), (2, 3)]  # left -> right across x = 0.5, normal u
        pairs_y = [(3, 0), (2, 1)]  # bottom -> top across y = 0.5, normal v
        ok, compressive = True, False
        for a, b in pairs_x:
            sa, sb = (q[a, 0], q[a, 1], 0, q[a, 3]), (q[b, 0], q[b, 1], 0, q[b, 3])
            ok &= _no_vacuum(sa, sb, gamma)
            compressive |= q[b, 1] < q[a, 1]
        for a, b in pairs_y:
            sa, sb = (q[a, 0], q[a, 2], 0, q[a, 3]), (q[b, 0], q[b, 2], 0, q[b, 3])
            ok &= _no_vacuum(sa, sb, gamma)
            compressive |= q[b, 2] < q[a, 2]
        if ok and compressive:
            return q


def four_quadrant_2d(nx, ny, seed, gamma=GAMMA, quads=None):
    """2D four-quadrant Riemann problem on [0,1]^2, split at x = y = 0.5.
    Returns (U[4,1,ny,nx], dx, quads).  dx = 1/nx (square cells, ny*dx need
    not be 1 for ragged test shapes)."""
    rng = np.random.default_rng(seed)
    if quads is None:
        quads = random_quadrants(rng, gamma)
    dx = 1.0 / nx
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * (1.0 / ny)
    X, Y = np.meshgrid(x, y)  # [ny, nx]
    idx = np.where(X >= 0.5, np.where(Y >= 0.5, 0, 3), np.where(Y >= 0.5, 1, 2))
    rho, u, v, p = (quads[idx, k] for k in range(4))
    return conserved(rho, [u, v], p, gamma).reshape(4, 1, ny, nx), dx, quads


def random_two_state(rng, gamma=GAMMA):
    """Random (rho, u, p) pair with the same ranges and vacuum rejection."""
    while True:
        a = (rng.uniform(0.1, 1.5), rng.uniform(-1, 1), 0.0, rng.uniform(0.03, 1.5))
        b = (rng.uniform(0.1, 1.5), rng.uniform(-1, 1), 0.0, rng.uniform(0.03, 1.5))
        if _no_vacuum(a, b, gamma):
            return (a[0], a[1], a[3]), (b[0], b[1], b[3])


# ----------------------------------------------------------------------------- 3D
def turbulence_3d(n, seed, mach=0.6, k0=4.0, gamma=GAMMA, ny=None, nz=None):
    """Decaying-turbulence initial field on [0, 2pi)^3, periodic.

    Solenoidal random-phase velocity with energy spectrum
    E(k) ~ k^4 exp(-2 (k/k0)^2), projected divergence-free in Fourier space,
    scaled to unit rms speed sqrt(<u.u>) = 1; rho = 1; uniform p with sound
    speed c = 1/mach so the turbulent Mach number is `mach`.
    Returns (U[5,nz,ny,nx], dx).  Non-cubic shapes keep dx = 2pi/n.
    """
    nx = n
    ny = ny or n
    nz = nz or n
    rng = np.random.default_rng(seed)
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    KX, KY, KZ = np.meshgrid(kx, ky, kz, indexing="ij")
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    K = np.sqrt(K2)
    # per-mode amplitude sqrt(E(k) / k^2) for a shell spectrum E(k)
    amp = np.where(K > 0, K * np.exp(-(K / k0) ** 2), 0.0)
    comps = [amp * np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, K.shape)) for _ in range(3)]
    # divergence-free projection: u_hat -= k (k . u_hat) / |k|^2
    kd = (KX * comps[0] + KY * comps[1] + KZ * comps[2]) / np.where(K2 > 0, K2, 1.0)
    comps = [comps[0] - KX * kd, comps[1] - KY * kd, comps[2] - KZ * kd]
    del KX, KY, KZ, K2, K, amp, kd
    # the real part of a solenoidal complex field is solenoidal
    vel = [np.fft.ifftn(c).real for c in comps]  # indexed [x, y, z]
    del comps
    urms = math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)))
    vel = [v / urms for v in vel]
    c = 1.0 / mach
    rho = np.ones((nx, ny, nz))
    p = rho * c * c / gamma
    U = conserved(rho, vel, p, gamma)  # [5, x, y, z]
    U = np.ascontiguousarray(U.transpose(0, 3, 2, 1))  # -> [5, z, y, x]
    return U, 2.0 * np.pi / n


# -------------------------------------------------------------------- serving
@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    shape: tuple            # (nx, ny, nz)
    dx: float
    U0: np.ndarray = field(repr=False)
    t_end: float = 0.0
    target_steps: int = 0


def request_stream(n_req=1024, rate=200.0, seed=0, frac_1d=0.7, n1d=(128, 8192),
                   n2d=(64, 512), steps=(50, 2000), gamma=GAMMA, cfl=0.5):
    """Poisson stream of independent Riemann runs of uneven sizes.

    70% 1D (N log-uniform in n1d, random two-state at x = 0.5), 30% 2D (side
    log-uniform in n2d, random four-quadrant state).  t_end is chosen from a
    target step count log-uniform in `steps`, using the largest initial signal
    speed |u| + sqrt(gamma p / rho) of the piecewise-constant data as the
    step-size estimate (an end-time recipe, not the solver's time step).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n_req):
        t += rng.exponential(1.0 / rate)
        nsteps = int(round(math.exp(rng.uniform(math.log(steps[0]), math.log(steps[1])))))
        if rng.uniform() < frac_1d:
            n = int(round(math.exp(rng.uniform(math.log(n1d[0]), math.log(n1d[1])))))
            left, right = random_two_state(rng, gamma)
            U0, dx = riemann_1d(n, left, right)
            smax = max(abs(s[1]) + math.sqrt(gamma * s[2] / s[0]) for s in (left, right))
            shape = (n, 1, 1)
        else:
            n = int(round(math.exp(rng.uniform(math.log(n2d[0]), math.log(n2d[1])))))
            U0, dx, q = four_quadrant_2d(n, n, int(rng.integers(1 << 31)), gamma)
            smax = max(abs(r[1]) + abs(r[2]) + 2 * math.sqrt(gamma * r[3] / r[0]) for r in q)
            shape = (n, n, 1)
        t_end = nsteps * cfl * dx / smax
        out.append(Request(rid, t, shape, dx, U0, t_end, nsteps))
    return out
