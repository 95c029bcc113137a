// Small kernels around the sweeps: CFL reduction and time-step finalisation,
// global Lax-Friedrichs speeds, and the per-face detector readback.
#pragma once
#include "wl2_device.hpp"

namespace wl2 {

constexpr int RED_BLOCK = 256;

// Block maximum of non-negative values; NaN propagates (any NaN wins).
__device__ __forceinline__ double block_max(double v, double* sh) {
  const bool nan = (v != v);
  v = wave_max(nan ? __longlong_as_double(0x7ff0000000000000LL) : v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
  }
  __syncthreads();
  return r;
}

// max over cells of sum_d (|u_d| + c) (cfl_speed: the operation order of the
// definition dt = cfl dx / max_cells sum_d (|u_d| + c), reproducible bit for
// bit).  Non-physical cells set status.
template <int NV>
__global__ __launch_bounds__(RED_BLOCK) void cfl_reduce_kernel(const double* __restrict__ U,
                                                               long long ncell, double gamma,
                                                               StepCtl* ctl) {
#pragma clang fp contract(off)
  constexpr int DIM = NV - 2;
  __shared__ double sh[RED_BLOCK / 64];
  double smax = 0.0;
  bool bad = false;
  for (long long c = (long long)blockIdx.x * RED_BLOCK + threadIdx.x; c < ncell;
       c += (long long)gridDim.x * RED_BLOCK) {
    double m[DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k) m[k] = U[(1 + k) * ncell + c];
    smax = nan_max(smax, cfl_speed<DIM>(U[c], m, U[(NV - 1) * ncell + c], gamma, bad));
  }
  const double bm = block_max(smax, sh);
  if (threadIdx.x == 0) {
    if (bm > 0.0 || bm != bm) cfl_fold(ctl, bm);
  }
  if (bad) atomicOr(&ctl->status, 1u);
}

// dt = cfl dx / smax (or a fixed dt), clipped to the device clock when
// use_clock (dt = 0, a no-op step, once the clock has reached t_end or a
// non-physical state was seen); resets the running maximum for the next
// reduction.  Launched as one wavefront.
[[maybe_unused]] static __global__ void finalize_dt_kernel(StepCtl* ctl, double cfl_dx, double dt_fixed, int use_clock,
                                          double s_floor) {
  if (blockIdx.x != 0 || threadIdx.x >= 64) return;
  double smax = cfl_take_wave(ctl);  // also resets it for the next reduction
  // speeds that enter through an inflow side (a NaN maximum stays NaN)
  if (s_floor > smax) smax = s_floor;
  if (threadIdx.x != 0) return;
  double dt = dt_fixed > 0.0 ? dt_fixed : cfl_dx / smax;
  ctl->t0 = ctl->t;  // the stages of the step run at t0, t0 + dt, t0 + dt/2
  if (use_clock) {
    // the clock stops at t_end and at the first non-physical state
    const double t = ctl->t, te = ctl->t_end;
    if (!(t < te) || ctl->status != 0u) {
      dt = 0.0;
    } else {
      if (t + dt > te) dt = te - t;
      ctl->t = t + dt;
      ctl->steps += 1u;
    }
  }
  ctl->dt = dt;
}

// State ghosts of the y sides of a 2D grid (Sec. 4.5: the double Mach
// reflection), for one stage: layer k of the low side is row -1-k, of the
// high side row ny+k.  STATE_WALL: bstate[0] under cells centred left of
// geom[0], the mirror image of the interior (y momentum negated) elsewhere;
// STATE_FRONT: bstate[0] left of the front x = geom[1] + geom[2] y +
// geom[3] t, bstate[1] right of it, at the stage time t = t0 + tc dt (tc <
// 0: the clock's t, for a right-hand side outside a step).  One thread per
// (side, layer, column).
struct YGhostRule {
  double state[2][4];
  double geom[4];
};

// Ghost value i of the 2 x 3 x nx (side, layer, column) of the y sides.
__device__ __forceinline__ void ghost_fill_item(const double* __restrict__ U, const KGrid& g,
                                                const StepCtl* ctl, double tc, double dx,
                                                const YGhostRule& rule, double* lo, double* hi,
                                                long long i) {
  const long long nx = g.n[0], ny = g.n[1];
  const int side = (int)(i / (3 * nx));
  const int layer = (int)((i / nx) % 3);
  const long long x = i % nx;
  const int kind = side ? g.bc_hi[1] : g.bc_lo[1];
  double* b = side ? hi : lo;
  if (kind < BC_STATE_WALL || b == nullptr) return;
  const double xc = ((double)x + 0.5) * dx;
  double u[4];
  if (kind == BC_STATE_FRONT) {
    const double t = tc < 0.0 ? ctl->t : ctl->t0 + tc * ctl->dt;
    const double yc = ((double)(side ? ny + layer : -1 - layer) + 0.5) * dx;
    const int s = xc < rule.geom[1] + rule.geom[2] * yc + rule.geom[3] * t ? 0 : 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) u[v] = rule.state[s][v];
  } else if (xc < rule.geom[0]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) u[v] = rule.state[0][v];
  } else {
    const long long row = side ? ny - 1 - layer : layer;
#pragma unroll
    for (int v = 0; v < 4; ++v) u[v] = U[v * g.ncell + row * nx + x];
    u[2] = -u[2];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) b[((long long)layer * 4 + v) * nx + x] = u[v];
}

[[maybe_unused]] static __global__ void ghost_fill_kernel(const double* __restrict__ U, KGrid g,
                                                          const StepCtl* ctl, double tc, double dx,
                                                          YGhostRule rule, double* lo, double* hi) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= 2 * 3 * (long long)g.n[0]) return;
  ghost_fill_item(U, g, ctl, tc, dx, rule, lo, hi, i);
}

// Program the device clock target (enqueued, no host synchronisation) and
// clear the running CFL maximum.
[[maybe_unused]] static __global__ void set_t_end_kernel(StepCtl* ctl, double t_end) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->t_end = t_end;
    cfl_clear(ctl);  // a maximum left by an earlier call is stale
  }
}

// Global LF speeds along every active direction: max over cells of
// |u_d - c|, |u_d|, |u_d + c| (fields u-c, entropy/shear, u+c), folded into
// the block's slot of ctl->lf_slots.  fmax passes over a NaN speed, as the
// oracle's comparison does (a non-physical cell stops the run through the
// CFL status instead).  GHOST: the same launch also fills the ghost rows of
// the y state sides of this stage (ghost_fill_item), which the speeds do
// not read.
template <int NV, bool GHOST>
__global__ __launch_bounds__(RED_BLOCK) void lf_reduce_kernel(const double* __restrict__ U,
                                                              long long ncell, double gamma,
                                                              StepCtl* ctl, KGrid g, double tc,
                                                              double dx, YGhostRule rule,
                                                              double* lo, double* hi) {
  constexpr int DIM = NV - 2;
  __shared__ double sh[RED_BLOCK / 64][3 * DIM];
  if (GHOST) {
    const long long ng = 2 * 3 * (long long)g.n[0];
    for (long long i = (long long)blockIdx.x * RED_BLOCK + threadIdx.x; i < ng;
         i += (long long)gridDim.x * RED_BLOCK)
      ghost_fill_item(U, g, ctl, tc, dx, rule, lo, hi, i);
  }
  double mx[DIM][3];
#pragma unroll
  for (int d = 0; d < DIM; ++d) mx[d][0] = mx[d][1] = mx[d][2] = 0.0;
  for (long long c = (long long)blockIdx.x * RED_BLOCK + threadIdx.x; c < ncell;
       c += (long long)gridDim.x * RED_BLOCK) {
    const double rho = U[c], E = U[(NV - 1) * ncell + c];
    const double ir = 1.0 / rho;
    double vel[DIM], mu = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      vel[k] = U[(1 + k) * ncell + c] * ir;
      mu += U[(1 + k) * ncell + c] * vel[k];
    }
    const double p = (gamma - 1.0) * (E - 0.5 * mu);
    const double cs = sqrt(gamma * p * ir);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      mx[d][0] = fmax(mx[d][0], fabs(vel[d] - cs));
      mx[d][1] = fmax(mx[d][1], fabs(vel[d]));
      mx[d][2] = fmax(mx[d][2], fabs(vel[d] + cs));
    }
  }
  // the 3 DIM block maxima in one exchange through LDS
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double w = wave_max(mx[d][j]);
      if (lane == 0) sh[wid][3 * d + j] = w;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 3 * DIM) {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < RED_BLOCK / 64; ++i) r = fmax(r, sh[i][t]);
    atomicMax(&ctl->lf_slots[blockIdx.x % LF_SLOTS].bits[t / 3][t % 3],
              (unsigned long long)__double_as_longlong(r));
  }
}

// The maximum over the slots into lf_bits (|u - c| for field 0, |u| for the
// entropy and shear fields, |u + c| for field nv - 1; directions beyond the
// grid's get 0) and the slots cleared for the next reduction.  One wave.
[[maybe_unused]] static __global__ void lf_finalize_kernel(StepCtl* ctl, int nv) {
  const int t = threadIdx.x;
  if (t < 9) {
    const int d = t / 3, j = t % 3;
    unsigned long long m = 0ull;
    for (int s = 0; s < LF_SLOTS; ++s) {
      const unsigned long long b = ctl->lf_slots[s].bits[d][j];
      m = b > m ? b : m;
      ctl->lf_slots[s].bits[d][j] = 0ull;
    }
    if (j == 0) ctl->lf_bits[d][0] = m;
    else if (j == 2) ctl->lf_bits[d][nv - 1] = m;
    else
      for (int k = 1; k < nv - 1; ++k) ctl->lf_bits[d][k] = m;
  }
}

// One thread per face along DIR: switch flags and detector values.
template <int NV, int DIR>
__global__ __launch_bounds__(256) void face_debug_kernel(const double* __restrict__ U, KGrid g,
                                                         KPhys ph, unsigned char* __restrict__ flags,
                                                         double* __restrict__ sigma,
                                                         long long nface) {
  const long long id = (long long)blockIdx.x * 256 + threadIdx.x;
  if (id >= nface) return;
  int fn[3] = {g.n[0], g.n[1], g.n[2]};
  fn[DIR] += 1;
  const int x = (int)(id % fn[0]);
  const int y = (int)((id / fn[0]) % fn[1]);
  const int z = (int)(id / ((long long)fn[0] * fn[1]));
  int ci[3] = {x, y, z};
  const int f = ci[DIR];
  ci[DIR] = 0;
  const long long base = ci[0] + (long long)ci[1] * g.stride[1] + (long long)ci[2] * g.stride[2];
  CellRec<NV> c[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double u[NV];
    load_state<NV, DIR>(U, g, base, f - 3 + m, u);
    make_rec<NV, DIR>(u, ph, c[m]);
  }
  double sig[NV];
  const unsigned weno = face_detector<NV, DIR>(c[0], c[1], c[2], c[3], c[4], c[5], ph,
                                               ph.eps_thr[DIR], sig);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    flags[k * nface + id] = ((weno >> k) & 1u) ? 0 : 1;
    sigma[k * nface + id] = sig[k];
  }
}

}  // namespace wl2
