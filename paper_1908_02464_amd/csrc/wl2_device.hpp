// Device-side arithmetic of the L2-norm regularized incremental-stencil WENO
// scheme (Zhu & Hu, arXiv 1908.02464) for the Euler equations, gfx950, FP64.
//
// Formulation used on the device (algebraically identical to the paper's
// steps, arranged for few FP64 instructions):
//  * Per cell, once per sweep: 1/rho, p, c, 1/sqrt(rho) and the flux F_d
//    along the sweep direction (Eq.(17)-(18)).
//  * Roe average (Sec. 2.3 step (1)) from the sqrt(rho) weights:
//    w u = m / sqrt(rho), w H = (E + p) / sqrt(rho); 1/rho~ = product of the
//    two 1/sqrt(rho), so the detector needs no division.
//  * Left eigenvectors (step (2)) are never stored: L x is evaluated as
//      K = u~ . m(x),  X = b2 x_rho + b1 (x_E - K),  Y = (u~_n x_rho - x_n)/c~
//      (u-c): (X + Y)/2   entropy: x_rho - X   shear t: (x_t - u~_t x_rho)/c~
//      (u+c): (X - Y)/2
//    with b1 = (gamma-1)/c~^2, b2 = b1 |u~|^2/2, and R f likewise from
//    S = f_{u-c} + f_0 + f_{u+c}.  Acoustic/entropy right eigenvectors have
//    unit density component, shear ones are scaled by c~.
//  * Linear branch (Eq.(34)): because sum_s R^s L^s = I, the face flux is
//      F = Fc6 + R delta,  delta^s = alpha^s dv^s                 (linear s)
//                          delta^s = f^s_WENO - L^s Fc6            (WENO s)
//    with Fc6 the six-point central flux and dv = L dU5 / 60 the detector
//    difference of Eq.(31).  The WENO part is added as a correction after
//    the linear sweep so the common (smooth) path stays short.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wl2 {

enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2, BC_INFLOW = 3,
       BC_STATE_WALL = 4, BC_STATE_FRONT = 5 };
enum { SPLIT_LLF = 0, SPLIT_LF = 1, SPLIT_ROE = 2 };
enum { HYB_PER_FIELD = 0, HYB_PER_FACE = 1, HYB_WENO_ONLY = 2, HYB_LINEAR_ONLY = 3 };
// weights of the WENO branch: regularized Eq.(28), original WENO-IS Eq.(8),
// WENO-IS with beta_01 on the 2-point stencils Eq.(14)-(15)
enum { W_L2IS = 0, W_IS = 1, W_IS_B01 = 2 };
// What a stage kernel does with the face-flux difference dU of Eq.(19):
// write it, add it to the output, or fuse it into the SSP-RK3 combination.
enum { OUT_WRITE = 0, OUT_ACCUM = 1, OUT_RK = 2 };

// Grid description passed by value to every kernel.
struct KGrid {
  int n[3];            // nx, ny, nz
  long long stride[3]; // element stride of one step along x, y, z
  long long ncell;     // nx*ny*nz, the stride between variables
  int bc_lo[3], bc_hi[3];
  // x- inflow side: the conserved state of the three ghosts of each x line,
  // [nvar][ny*nz] (null for every other boundary rule)
  const double* inflow;
  // y sides of a 2D grid with state ghosts (BC_STATE_WALL, BC_STATE_FRONT):
  // their three ghost rows, [layer][nvar][nx] (layer 0 next to the grid),
  // filled before every stage by ghost_fill_kernel (null otherwise)
  const double* ygh[2];
};

// Physical and scheme constants passed by value.
struct KPhys {
  double gamma, gm1, dx, inv_dx, cfl;
  double c_reg, eps_w;
  double eps_thr[3];   // switch threshold C (dx/L_d)^alpha per direction
  int split, hybrid;
  int weights;         // W_*: weights of the WENO branch
};

// One slot of the running CFL maximum (max of sum_d(|u_d|+c) as raw bits;
// the values are >= 0, so their bit patterns order like the values), alone
// in its 128-byte line.  The waves of a launch fold into CFL_SLOTS different
// lines, so that their atomics do not queue on one address.
constexpr int CFL_SLOTS = 32;
struct alignas(128) CflSlot {
  unsigned long long bits;
};

// Global Lax-Friedrichs speeds: the blocks of the reduction fold their
// maxima into LF_SLOTS slots (block b into slot b mod LF_SLOTS), each in its
// own 128-byte line, so that their atomics do not queue on one address (on
// one line, 2048 blocks x 8 atomics took 34 us at 1024^2); a one-wave kernel
// then takes the maximum over the slots into lf_bits and clears them.
constexpr int LF_SLOTS = 16;
struct alignas(128) LfSlot {
  unsigned long long bits[3][3];  // direction, (|u - c|, |u|, |u + c|) maxima (raw bits)
};

// Device control block of one grid (time step, clock, status).
struct StepCtl {
  unsigned int status;           // sticky: bit 0 = non-physical state seen
  unsigned int steps;            // clock steps taken (steps that advanced t)
  double dt;                     // dt of the step in flight
  double t;                      // simulated time after the step in flight
  double t0;                     // simulated time at the start of the step in flight
  double t_end;                  // > 0: clip the clock to it
  unsigned long long lf_bits[3][5];  // global LF speeds (raw bits) per direction, field
  unsigned int list_n[2];        // entries in the nonlinear-correction list: consecutive
                                 // stages alternate between the two counters, and each
                                 // stage's correction kernel clears the next one's
  CflSlot smax[CFL_SLOTS];       // running CFL maximum, spread over slots
  LfSlot lf_slots[LF_SLOTS];     // global LF speeds being reduced (zero between reductions)
};

// Fold a maximum (> 0, or +inf standing for NaN) into the wave's slot.
__device__ __forceinline__ void cfl_fold(StepCtl* ctl, double m) {
  const unsigned wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  atomicMax(&ctl->smax[wave % CFL_SLOTS].bits, (unsigned long long)__double_as_longlong(m));
}

// Clear the running maximum (one thread).
__device__ __forceinline__ void cfl_clear(StepCtl* ctl) {
#pragma unroll
  for (int s = 0; s < CFL_SLOTS; ++s) ctl->smax[s].bits = 0ull;
}

// The running maximum over all slots, which are cleared for the next
// reduction (one thread, after the folding launches have finished).
__device__ __forceinline__ double cfl_take(StepCtl* ctl) {
  unsigned long long m = 0ull;
#pragma unroll
  for (int s = 0; s < CFL_SLOTS; ++s) {
    const unsigned long long b = ctl->smax[s].bits;
    m = b > m ? b : m;
  }
  cfl_clear(ctl);
  return __longlong_as_double((long long)m);
}

// The running maximum over all slots read by one whole wavefront (lane s
// reads slot s; every lane gets the maximum), the slots left as they are.
__device__ __forceinline__ double cfl_peek_wave(const StepCtl* ctl) {
  static_assert(CFL_SLOTS <= 64, "one slot per lane");
  const int lane = threadIdx.x & 63;
  unsigned long long m = lane < CFL_SLOTS ? ctl->smax[lane].bits : 0ull;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long q = __shfl_xor(m, o, 64);
    m = q > m ? q : m;
  }
  return __longlong_as_double((long long)m);
}

// cfl_take by one whole wavefront (lane s reads and clears slot s): one
// round trip to memory instead of CFL_SLOTS.  Every lane gets the maximum.
__device__ __forceinline__ double cfl_take_wave(StepCtl* ctl) {
  static_assert(CFL_SLOTS <= 64, "one slot per lane");
  const int lane = threadIdx.x & 63;
  unsigned long long m = 0ull;
  if (lane < CFL_SLOTS) {
    m = ctl->smax[lane].bits;
    ctl->smax[lane].bits = 0ull;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long q = __shfl_xor(m, o, 64);
    m = q > m ? q : m;
  }
  return __longlong_as_double((long long)m);
}

// The device-clock dt of a step from the CFL maximum folded by the step
// before, by finalize_dt_kernel's rule, formed by every wavefront of a
// stage-1 kernel itself (all of its lanes call; every wavefront reads the
// same slots and clock, so gets the same bits).  The lane with writer set
// records t0 = t, dt and the step count; it leaves t and the slots alone,
// which other wavefronts still read: the stage's correction kernel sets
// t = t0 + dt (the same value as t + dt) and clears the slots
// (clock_commit).
__device__ __forceinline__ double clock_dt_wave(StepCtl* ctl, double cfl_dx, double s_floor,
                                                bool writer) {
  double smax = cfl_peek_wave(ctl);
  if (s_floor > smax) smax = s_floor;
  double dt = cfl_dx / smax;
  const double t = ctl->t, te = ctl->t_end;
  const bool stop = !(t < te) || ctl->status != 0u;
  if (stop) dt = 0.0;
  else if (t + dt > te) dt = te - t;
  if (writer) {
    ctl->t0 = t;
    ctl->dt = dt;
    if (!stop) ctl->steps += 1u;
  }
  return dt;
}

// After every wavefront of the stage-1 kernel has read the clock: t = t0 +
// dt (t itself when the clock stopped, dt = 0) and the CFL slots cleared for
// the step's own fold (one thread).
__device__ __forceinline__ void clock_commit(StepCtl* ctl) {
  ctl->t = ctl->t0 + ctl->dt;
  cfl_clear(ctl);
}

// ---------------------------------------------------------------- CFL
// Signal speed sum_d (|u_d| + c) of one cell, in the operation order of the
// time-step definition (correctly rounded division and square root, no
// contraction), so every kernel that reduces it gets the same bits; sets
// bad for a non-finite or non-physical (rho <= 0 or p <= 0) state.
template <int DIM>
__device__ __forceinline__ double cfl_speed(double rho, const double (&m)[DIM], double E,
                                            double gamma, bool& bad) {
#pragma clang fp contract(off)
  double vel[DIM], q = 0.0;
  bool fin = isfinite(rho) && isfinite(E);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    fin = fin && isfinite(m[k]);
    vel[k] = m[k] / rho;
    q += vel[k] * vel[k];
  }
  q *= 0.5;
  const double p = (gamma - 1.0) * (E - rho * q);
  const double cs = sqrt(gamma * p / rho);
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) s += fabs(vel[k]) + cs;
  if (!fin || !(rho > 0.0) || !(p > 0.0)) bad = true;
  return s;
}

// cfl_speed of a conserved state u = (rho, momentum, E).
template <int NV>
__device__ __forceinline__ double cfl_speed_u(const double (&u)[NV], double gamma, bool& bad) {
  double m[NV - 2];
#pragma unroll
  for (int k = 0; k < NV - 2; ++k) m[k] = u[1 + k];
  return cfl_speed<NV - 2>(u[0], m, u[NV - 1], gamma, bad);
}

// Running maximum that lets a NaN win.
__device__ __forceinline__ double nan_max(double acc, double s) { return (s != s || s > acc) ? s : acc; }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Fold one wave's CFL maximum and non-physical flag into the step control
// word (one atomic per wave; a NaN maximum is raised to +inf so that it
// wins).  Every lane of the wave must call it.
__device__ __forceinline__ void cfl_commit_wave(StepCtl* ctl, double smax, bool bad) {
  const bool nan = (smax != smax);
  const double m = wave_max(nan ? __longlong_as_double(0x7ff0000000000000LL) : smax);
  const unsigned long long anybad = __ballot(bad);
  if ((threadIdx.x & 63) == 0) {
    if (m > 0.0) cfl_fold(ctl, m);
    if (anybad) atomicOr(&ctl->status, 1u);
  }
}

// ---------------------------------------------------------------- ghosts
// Interior index for a line position k in [-3, n+2]; *flip = 1 when the
// ghost is a mirror image whose normal momentum changes sign.
__device__ __forceinline__ int ghost_index(int k, int n, int lo, int hi, bool& flip) {
  flip = false;
  if (k >= 0 && k < n) return k;
  if (k < 0) {
    if (lo == BC_PERIODIC) { int r = k % n; return r < 0 ? r + n : r; }
    // inflow and state ghosts are taken from KGrid::inflow / ygh by the
    // caller; the index returned is an in-grid one
    if (lo == BC_TRANSMISSIVE || lo == BC_INFLOW || lo >= BC_STATE_WALL) return 0;
    flip = true;
    return -1 - k;
  }
  if (hi == BC_PERIODIC) return k % n;
  if (hi == BC_TRANSMISSIVE || hi >= BC_STATE_WALL) return n - 1;
  flip = true;
  return 2 * n - 1 - k;
}

// Is line position y (outside 0..ny-1) a state ghost of a y side?
__device__ __forceinline__ bool is_yghost(const KGrid& g, int y) {
  return (y < 0 && g.bc_lo[1] >= BC_STATE_WALL) || (y >= g.n[1] && g.bc_hi[1] >= BC_STATE_WALL);
}

// State ghost at column x, row y (outside the grid) of a 2D grid.
template <int NV>
__device__ __forceinline__ void load_yghost(const KGrid& g, long long x, int y, double (&u)[NV]) {
  const int side = y < 0 ? 0 : 1;
  int layer = y < 0 ? -1 - y : y - g.n[1];
  layer = layer > 2 ? 2 : layer;
  const double* b = g.ygh[side] + (long long)layer * NV * g.n[0];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = b[(long long)v * g.n[0] + x];
}

// Ghost state of the x- inflow side for x line `row` (= y + ny*z).
template <int NV>
__device__ __forceinline__ void load_inflow(const KGrid& g, long long row, double (&u)[NV]) {
  const long long rows = (long long)g.n[1] * g.n[2];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = g.inflow[v * rows + row];
}

// Load the conserved state at line position k along DIR of the line whose
// cell 0 is at element offset `base`.
template <int NV, int DIR>
__device__ __forceinline__ void load_state(const double* __restrict__ U, const KGrid& g,
                                           long long base, int k, double (&u)[NV]) {
  bool flip;
  const int idx = ghost_index(k, g.n[DIR], g.bc_lo[DIR], g.bc_hi[DIR], flip);
  const long long off = base + (long long)idx * g.stride[DIR];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = U[v * g.ncell + off];
  if (flip) u[1 + DIR] = -u[1 + DIR];
  // x lines start at cell offset row * nx
  if (DIR == 0 && k < 0 && g.bc_lo[0] == BC_INFLOW) load_inflow<NV>(g, base / g.n[0], u);
  // y lines of a 2D grid start at cell offset x
  if (DIR == 1 && NV == 4 && (k < 0 || k >= g.n[1]) && is_yghost(g, k)) load_yghost<NV>(g, base, k, u);
}

// ---------------------------------------------------------------- cells
template <int NV>
struct CellRec {
  double U[NV];  // conserved state
  double F[NV];  // physical flux along the sweep direction
  double un;     // normal velocity
  double c;      // sound speed
  double iw;     // 1/sqrt(rho)
  double p;      // pressure
};

template <int NV, int DIR>
__device__ __forceinline__ void make_rec(const double (&u)[NV], const KPhys& ph, CellRec<NV>& r) {
  constexpr int DIM = NV - 2;
  const double rho = u[0], E = u[NV - 1];
  const double ir = 1.0 / rho;
  double vel[DIM];
  double mu = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    vel[k] = u[1 + k] * ir;
    mu += u[1 + k] * vel[k];
  }
  const double p = ph.gm1 * (E - 0.5 * mu);
  r.c = sqrt(ph.gamma * p * ir);
  r.iw = sqrt(ir);
  r.p = p;
  r.un = vel[DIR];
  const double mn = u[1 + DIR];
#pragma unroll
  for (int v = 0; v < NV; ++v) r.U[v] = u[v];
  r.F[0] = mn;
#pragma unroll
  for (int k = 0; k < DIM; ++k) r.F[1 + k] = mn * vel[k] + (k == DIR ? p : 0.0);
  r.F[NV - 1] = (E + p) * vel[DIR];
}

// ---------------------------------------------------------------- Roe state
template <int NV>
struct Roe {
  double u[NV - 2];
  double H, c, ic, q, b1, b2, irho;
};

template <int NV, int DIR>
__device__ __forceinline__ void roe_average(const CellRec<NV>& L, const CellRec<NV>& R,
                                            const KPhys& ph, Roe<NV>& s) {
  constexpr int DIM = NV - 2;
  const double wl = L.U[0] * L.iw, wr = R.U[0] * R.iw;
  const double is = 1.0 / (wl + wr);
  double q = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    s.u[k] = (L.U[1 + k] * L.iw + R.U[1 + k] * R.iw) * is;
    q += s.u[k] * s.u[k];
  }
  s.q = 0.5 * q;
  s.H = ((L.U[NV - 1] + L.p) * L.iw + (R.U[NV - 1] + R.p) * R.iw) * is;
  s.c = sqrt(ph.gm1 * (s.H - s.q));
  s.ic = 1.0 / s.c;
  s.b1 = ph.gm1 * s.ic * s.ic;
  s.b2 = s.b1 * s.q;
  s.irho = L.iw * R.iw;  // 1 / sqrt(rho_L rho_R)
}

// out = L x   (field order: u-c, entropy, shear..., u+c)
template <int NV, int DIR>
__device__ __forceinline__ void project(const Roe<NV>& s, const double (&x)[NV], double (&o)[NV]) {
  constexpr int DIM = NV - 2;
  double K = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) K += s.u[k] * x[1 + k];
  const double X = s.b2 * x[0] + s.b1 * (x[NV - 1] - K);
  const double Y = (s.u[DIR] * x[0] - x[1 + DIR]) * s.ic;
  o[0] = 0.5 * (X + Y);
  o[1] = x[0] - X;
  int f = 2;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    if (k == DIR) continue;
    o[f++] = (x[1 + k] - s.u[k] * x[0]) * s.ic;
  }
  o[NV - 1] = 0.5 * (X - Y);
}

// out = R f
template <int NV, int DIR>
__device__ __forceinline__ void back_project(const Roe<NV>& s, const double (&f)[NV], double (&o)[NV]) {
  constexpr int DIM = NV - 2;
  const double a = f[0], b = f[1], g = f[NV - 1];
  const double S = a + b + g, D = s.c * (g - a);
  o[0] = S;
  double eE = s.H * (a + g) + s.u[DIR] * D + s.q * b;
  int fi = 2;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    if (k == DIR) {
      o[1 + k] = s.u[k] * S + D;
    } else {
      const double e = f[fi++];
      o[1 + k] = s.u[k] * S + s.c * e;
      eE += s.c * s.u[k] * e;
    }
  }
  o[NV - 1] = eE;
}

// ---------------------------------------------------------------- face
// Splitting speed per field.
template <int NV, int DIR>
__device__ __forceinline__ void split_speeds(const CellRec<NV>& c0, const CellRec<NV>& c1,
                                             const CellRec<NV>& c2, const CellRec<NV>& c3,
                                             const CellRec<NV>& c4, const CellRec<NV>& c5,
                                             const Roe<NV>& s, const KPhys& ph,
                                             const double* lf, double (&a)[NV]) {
  if (ph.split == SPLIT_LLF) {
    // max over the six stencil cells of |u_n - c|, |u_n|, |u_n + c|
    double am = fabs(c0.un - c0.c), a0 = fabs(c0.un), ap = fabs(c0.un + c0.c);
#define WL2_MX(C)                                 \
  am = fmax(am, fabs((C).un - (C).c));            \
  a0 = fmax(a0, fabs((C).un));                    \
  ap = fmax(ap, fabs((C).un + (C).c));
    WL2_MX(c1) WL2_MX(c2) WL2_MX(c3) WL2_MX(c4) WL2_MX(c5)
#undef WL2_MX
    a[0] = am;
#pragma unroll
    for (int k = 1; k < NV - 1; ++k) a[k] = a0;
    a[NV - 1] = ap;
  } else if (ph.split == SPLIT_ROE) {
    a[0] = fabs(s.u[DIR] - s.c);
#pragma unroll
    for (int k = 1; k < NV - 1; ++k) a[k] = fabs(s.u[DIR]);
    a[NV - 1] = fabs(s.u[DIR] + s.c);
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] = lf[k];
  }
}

// Linear-branch flux of one face (all fields as if linear) plus the switch
// decision.  Returns the bit mask of fields that need the WENO flux.
template <int NV, int DIR>
__device__ __forceinline__ unsigned face_linear(const CellRec<NV>& c0, const CellRec<NV>& c1,
                                                const CellRec<NV>& c2, const CellRec<NV>& c3,
                                                const CellRec<NV>& c4, const CellRec<NV>& c5,
                                                const KPhys& ph, double eps_thr, const double* lf,
                                                double (&Fh)[NV]) {
  Roe<NV> s;
  roe_average<NV, DIR>(c2, c3, ph, s);
  double dU5[NV], Fc6[NV];
  constexpr double k60 = 1.0 / 60.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    dU5[i] = (c0.U[i] - c5.U[i]) + 5.0 * (c4.U[i] - c1.U[i]) + 10.0 * (c2.U[i] - c3.U[i]);
    Fc6[i] = ((c0.F[i] + c5.F[i]) - 8.0 * (c1.F[i] + c4.F[i]) + 37.0 * (c2.F[i] + c3.F[i])) * k60;
  }
  double dv[NV];
  project<NV, DIR>(s, dU5, dv);
  double a[NV];
  split_speeds<NV, DIR>(c0, c1, c2, c3, c4, c5, s, ph, lf, a);
  unsigned weno = 0;
  double smax = 0.0;
  double d[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    dv[k] *= k60;
    const double t = dv[k] * s.irho;
    const double sig = t * t;  // Eq.(30)
    smax = fmax(smax, sig);
    if (!(sig < eps_thr)) weno |= 1u << k;
    d[k] = a[k] * dv[k];
  }
  if (ph.hybrid == HYB_PER_FACE) weno = (smax < eps_thr) ? 0u : ((1u << NV) - 1u);
  else if (ph.hybrid == HYB_WENO_ONLY) weno = (1u << NV) - 1u;
  else if (ph.hybrid == HYB_LINEAR_ONLY) weno = 0u;
  double Rd[NV];
  back_project<NV, DIR>(s, d, Rd);
#pragma unroll
  for (int i = 0; i < NV; ++i) Fh[i] = Fc6[i] + Rd[i];
  return weno;
}

// Detector values and decisions only (for the debug readback).
template <int NV, int DIR>
__device__ __forceinline__ unsigned face_detector(const CellRec<NV>& c0, const CellRec<NV>& c1,
                                                  const CellRec<NV>& c2, const CellRec<NV>& c3,
                                                  const CellRec<NV>& c4, const CellRec<NV>& c5,
                                                  const KPhys& ph, double eps_thr, double (&sig)[NV]) {
  Roe<NV> s;
  roe_average<NV, DIR>(c2, c3, ph, s);
  double dU5[NV], dv[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i)
    dU5[i] = (c0.U[i] - c5.U[i]) + 5.0 * (c4.U[i] - c1.U[i]) + 10.0 * (c2.U[i] - c3.U[i]);
  project<NV, DIR>(s, dU5, dv);
  unsigned weno = 0;
  double smax = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double t = dv[k] * (1.0 / 60.0) * s.irho;
    sig[k] = t * t;
    smax = fmax(smax, sig[k]);
    if (!(sig[k] < eps_thr)) weno |= 1u << k;
  }
  if (ph.hybrid == HYB_PER_FACE) weno = (smax < eps_thr) ? 0u : ((1u << NV) - 1u);
  else if (ph.hybrid == HYB_WENO_ONLY) weno = (1u << NV) - 1u;
  else if (ph.hybrid == HYB_LINEAR_ONLY) weno = 0u;
  return weno;
}

// ---------------------------------------------------------------- WENO-L2IS
// Scalar reconstruction at x_{j+1/2} from f_{j-2..j+2} (Eq.(5),(6),(11),
// (27),(28)), optimal weights d = (0.4, 0.2, 0.3, 0.1); wts selects the
// comparison weights of Eq.(8) or Eq.(14)-(15) instead (lam unused there).
__device__ __forceinline__ double weno_l2is(double fm2, double fm1, double f0, double fp1,
                                            double fp2, double lam, double eps_w, int wts) {
  const double q0 = 0.5 * (f0 + fp1);
  const double q1 = 0.5 * (3.0 * f0 - fm1);
  const double q2 = (2.0 * f0 + 5.0 * fp1 - fp2) * (1.0 / 6.0);
  const double q3 = (2.0 * fm2 - 7.0 * fm1 + 11.0 * f0) * (1.0 / 6.0);
  const double d0 = fp1 - f0, d1 = f0 - fm1;
  const double b0 = d0 * d0, b1 = d1 * d1;
  const double s2a = f0 - 2.0 * fp1 + fp2, s2b = 3.0 * f0 - 4.0 * fp1 + fp2;
  const double s3a = fm2 - 2.0 * fm1 + f0, s3b = fm2 - 4.0 * fm1 + 3.0 * f0;
  const double b2 = (13.0 / 12.0) * s2a * s2a + 0.25 * s2b * s2b;
  const double b3 = (13.0 / 12.0) * s3a * s3a + 0.25 * s3b * s3b;
  const double t1 = (fp2 + fm2) - 4.0 * (fp1 + fm1) + 6.0 * f0;
  const double t2 = (fp2 - fm2) - 2.0 * (fp1 - fm1);
  const double tau5 = (13.0 / 12.0) * t1 * t1 + 0.25 * t2 * t2;
  const double e = fm1 - 2.0 * f0 + fp1;
  double a0, a1, a2, a3;
  if (wts == W_L2IS) {
    const double E01 = e * e * (1.0 / 45.0);
    const double lt = lam * tau5;
    a0 = 0.4 * (1.0 + lt / (lam * b0 + E01 + eps_w));
    a1 = 0.2 * (1.0 + lt / (lam * b1 + E01 + eps_w));
    a2 = 0.3 * (1.0 + lt / (lam * b2 + eps_w));
    a3 = 0.1 * (1.0 + lt / (lam * b3 + eps_w));
  } else {
    double r0 = tau5 / (b0 + eps_w), r1 = tau5 / (b1 + eps_w);
    if (wts == W_IS_B01) {
      const double g = fm1 - fp1;
      const double r01 = tau5 / ((13.0 / 12.0) * e * e + 0.25 * g * g + eps_w);
      r0 *= r01;
      r1 *= r01;
    }
    a0 = 0.4 * (1.0 + r0);
    a1 = 0.2 * (1.0 + r1);
    a2 = 0.3 * (1.0 + tau5 / (b2 + eps_w));
    a3 = 0.1 * (1.0 + tau5 / (b3 + eps_w));
  }
  return (a0 * q0 + a1 * q1 + a2 * q2 + a3 * q3) / ((a0 + a1) + (a2 + a3));
}

// Row k of L (the left eigenvector of field k) as coefficients.
template <int NV, int DIR, int K>
__device__ __forceinline__ void left_row(const Roe<NV>& s, double (&r)[NV]) {
  constexpr int DIM = NV - 2;
  if (K == 0 || K == NV - 1) {
    const double sg = (K == 0) ? 1.0 : -1.0;
    r[0] = 0.5 * (s.b2 + sg * s.u[DIR] * s.ic);
#pragma unroll
    for (int k = 0; k < DIM; ++k) r[1 + k] = 0.5 * (-s.b1 * s.u[k] - (k == DIR ? sg * s.ic : 0.0));
    r[NV - 1] = 0.5 * s.b1;
  } else if (K == 1) {
    r[0] = 1.0 - s.b2;
#pragma unroll
    for (int k = 0; k < DIM; ++k) r[1 + k] = s.b1 * s.u[k];
    r[NV - 1] = -s.b1;
  } else {
    // shear field K-2: the (K-2)-th tangential momentum component
    int t = K - 2;
    int comp = (t < DIR) ? t : t + 1;
    r[0] = -s.u[comp] * s.ic;
#pragma unroll
    for (int k = 0; k < DIM; ++k) r[1 + k] = (k == comp) ? s.ic : 0.0;
    r[NV - 1] = 0.0;
  }
}

template <int NV>
__device__ __forceinline__ double dot(const double (&r)[NV], const double (&x)[NV]) {
  double a = r[0] * x[0];
#pragma unroll
  for (int i = 1; i < NV; ++i) a += r[i] * x[i];
  return a;
}

template <int NV, int DIR, int K>
__device__ __forceinline__ double weno_field(const CellRec<NV>& c0, const CellRec<NV>& c1,
                                             const CellRec<NV>& c2, const CellRec<NV>& c3,
                                             const CellRec<NV>& c4, const CellRec<NV>& c5,
                                             const Roe<NV>& s, double al, double dvk,
                                             double LFk, const KPhys& ph) {
  double r[NV];
  left_row<NV, DIR, K>(s, r);
  const double t = dvk * s.irho;
  const double lam = ph.c_reg * (t * t);  // Eq.(32)
  // f+-_m = (g_m +- alpha v_m)/2, v = L^K U_m, g = L^K F_m  (Eq.(20)-(21))
#define WL2_SPL(C, P, M)                        \
  {                                             \
    const double vv = dot<NV>(r, (C).U);        \
    const double gg = dot<NV>(r, (C).F);        \
    P = 0.5 * (gg + al * vv);                   \
    M = 0.5 * (gg - al * vv);                   \
  }
  double p0, p1, p2, p3, p4, p5, m0, m1, m2, m3, m4, m5;
  WL2_SPL(c0, p0, m0) WL2_SPL(c1, p1, m1) WL2_SPL(c2, p2, m2)
  WL2_SPL(c3, p3, m3) WL2_SPL(c4, p4, m4) WL2_SPL(c5, p5, m5)
#undef WL2_SPL
  (void)p5;
  (void)m0;
  // f+ on (f+_{j-2..j+2}); f- on the mirrored (f-_{j+3..j-1})  (Eq.(22)-(23))
  const double fw = weno_l2is(p0, p1, p2, p3, p4, lam, ph.eps_w, ph.weights) +
                    weno_l2is(m5, m4, m3, m2, m1, lam, ph.eps_w, ph.weights);
  return fw - (LFk + al * dvk);
}

// Correction R (f_WENO - f_lin) of one face for the fields in `mask`.  Added
// to the linear flux it gives the hybrid flux of Eq.(33) (per-field switch).
template <int NV, int DIR>
__device__ __forceinline__ void face_weno_correction(const CellRec<NV>& c0, const CellRec<NV>& c1,
                                                     const CellRec<NV>& c2, const CellRec<NV>& c3,
                                                     const CellRec<NV>& c4, const CellRec<NV>& c5,
                                                     unsigned mask, const KPhys& ph,
                                                     const double* lf, double (&dF)[NV]) {
  Roe<NV> s;
  roe_average<NV, DIR>(c2, c3, ph, s);
  double dU5[NV], Fc6[NV];
  constexpr double k60 = 1.0 / 60.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    dU5[i] = (c0.U[i] - c5.U[i]) + 5.0 * (c4.U[i] - c1.U[i]) + 10.0 * (c2.U[i] - c3.U[i]);
    Fc6[i] = ((c0.F[i] + c5.F[i]) - 8.0 * (c1.F[i] + c4.F[i]) + 37.0 * (c2.F[i] + c3.F[i])) * k60;
  }
  double dv[NV], LF[NV], a[NV];
  project<NV, DIR>(s, dU5, dv);
  project<NV, DIR>(s, Fc6, LF);
  split_speeds<NV, DIR>(c0, c1, c2, c3, c4, c5, s, ph, lf, a);
  double del[NV];
#define WL2_FIELD(K)                                                                   \
  if (K < NV) {                                                                        \
    del[K < NV ? K : 0] = 0.0;                                                         \
    if ((mask >> K) & 1u)                                                              \
      del[K < NV ? K : 0] = weno_field<NV, DIR, (K < NV ? K : 0)>(                     \
          c0, c1, c2, c3, c4, c5, s, a[K < NV ? K : 0], dv[K < NV ? K : 0] * k60,      \
          LF[K < NV ? K : 0], ph);                                                     \
  }
  WL2_FIELD(0) WL2_FIELD(1) WL2_FIELD(2) WL2_FIELD(3) WL2_FIELD(4)
#undef WL2_FIELD
  back_project<NV, DIR>(s, del, dF);
}

}  // namespace wl2
