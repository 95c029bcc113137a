// Kernels of the per-direction sweep path (gfx950, FP64).
//
// sweep_kernel: one thread walks a segment of S cells of one grid line along
// the sweep direction DIR with a six-cell window of per-cell records held in
// registers (the loop is fully unrolled so the window never moves).  Lanes of
// a wavefront take adjacent lines (y and z sweeps: adjacent x, so every load
// is a coalesced 512-byte row) or adjacent segments of one row (x sweep).
// Every face first gets the linear-branch flux; faces whose detector asks for
// the nonlinear flux in some field are corrected afterwards (the correction
// is linear in the face flux, so it can be added to the outputs of the two
// neighbouring cells owned by this thread).
// The output is the face-flux difference of Eq.(19), written, accumulated, or
// fused into the SSP-RK3 stage combination.
#pragma once
#include "wl2_device.hpp"

namespace wl2 {

struct SweepArgs {
  const double* Uk;    // stage input: the stencil source
  double* out;         // WRITE/ACCUM: dU/dt (or partial sum); RK: U^(k+1)
  const double* acc;   // RK: partial sum of the other directions (or null)
  const double* Un;    // RK: U^n (read when rk_a != 0)
  const StepCtl* ctl;  // dt (RK) and global LF speeds
  double rk_a, rk_b;   // RK: out = rk_a U^n + rk_b (Uk + dt (acc + dU))
};

constexpr int SWEEP_BLOCK = 256;

// Element offset of cell 0 of the line of thread `gid`, and its segment.
template <int DIR>
__device__ __forceinline__ void sweep_map(long long gid, const KGrid& g, int nseg, long long& base,
                                          int& seg) {
  if (DIR == 0) {
    seg = (int)(gid % nseg);
    base = (gid / nseg) * (long long)g.n[0];
  } else if (DIR == 1) {
    const int x = (int)(gid % g.n[0]);
    const long long r = gid / g.n[0];
    seg = (int)(r % nseg);
    const long long z = r / nseg;
    base = x + z * g.stride[2];
  } else {
    const int x = (int)(gid % g.n[0]);
    const long long r = gid / g.n[0];
    const int y = (int)(r % g.n[1]);
    seg = (int)(r / g.n[1]);
    base = x + (long long)y * g.n[0];
  }
}

// Work of one thread: segment `gid` (0 <= gid < nseg * lines) of the sweep
// along DIR.  Shared by the single-grid kernel and the batched kernel, so a
// grid gets the same bits whether it runs alone or in a batch.
template <int NV, int DIR, int S, int OUT>
__device__ __forceinline__ void sweep_body(const SweepArgs& a, const KGrid& g, const KPhys& ph,
                                           int nseg, long long gid) {
  long long base;
  int seg;
  sweep_map<DIR>(gid, g, nseg, base, seg);
  const int n = g.n[DIR];
  const int s0 = seg * S;
  const int cnt = min(S, n - s0);
  const long long st = g.stride[DIR];
  double dt = 0.0;
  if (OUT == OUT_RK) {
    dt = a.ctl->dt;
    if (!(dt > 0.0)) return;  // finished run: leave the state untouched
  }
  double lf[NV];
  if (ph.split == SPLIT_LF) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lf[k] = __longlong_as_double((long long)a.ctl->lf_bits[DIR][k]);
  }
  const double eps_thr = ph.eps_thr[DIR];
  const double scale = (OUT == OUT_RK) ? a.rk_b * dt : 1.0;

  CellRec<NV> w[6];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    double u[NV];
    load_state<NV, DIR>(a.Uk, g, base, s0 - 3 + m, u);
    make_rec<NV, DIR>(u, ph, w[m]);
  }
  double Fprev[NV];
  unsigned need = 0;
#pragma unroll
  for (int f = 0; f <= S; ++f) {
    if (f <= cnt) {
      {
        double u[NV];
        load_state<NV, DIR>(a.Uk, g, base, s0 + f + 2, u);
        make_rec<NV, DIR>(u, ph, w[(f + 5) % 6]);
      }
      double Fh[NV];
      const unsigned m = face_linear<NV, DIR>(w[f % 6], w[(f + 1) % 6], w[(f + 2) % 6],
                                               w[(f + 3) % 6], w[(f + 4) % 6], w[(f + 5) % 6],
                                               ph, eps_thr, lf, Fh);
      if (m) need |= 1u << f;
      if (f > 0) {
        const long long off = base + (long long)(s0 + f - 1) * st;
        const CellRec<NV>& cc = w[(f + 2) % 6];  // cell s0+f-1
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double dU = (Fprev[v] - Fh[v]) * ph.inv_dx;
          double* o = a.out + v * g.ncell + off;
          if (OUT == OUT_WRITE) {
            *o = dU;
          } else if (OUT == OUT_ACCUM) {
            *o += dU;
          } else {
            const double tot = a.acc ? a.acc[v * g.ncell + off] + dU : dU;
            double r = a.rk_b * (cc.U[v] + dt * tot);
            if (a.rk_a != 0.0) r += a.rk_a * a.Un[v * g.ncell + off];
            *o = r;
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Fprev[v] = Fh[v];
    }
  }
  // nonlinear corrections of the flagged faces
  while (need) {
    const int f = __builtin_ctz(need);
    need &= need - 1;
    CellRec<NV> c[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      double u[NV];
      load_state<NV, DIR>(a.Uk, g, base, s0 + f - 3 + m, u);
      make_rec<NV, DIR>(u, ph, c[m]);
    }
    unsigned mask;
    {
      double sig[NV];
      mask = face_detector<NV, DIR>(c[0], c[1], c[2], c[3], c[4], c[5], ph, eps_thr, sig);
    }
    double dF[NV];
    face_weno_correction<NV, DIR>(c[0], c[1], c[2], c[3], c[4], c[5], mask, ph, lf, dF);
    // face f lies between cells s0+f-1 (loses dF) and s0+f (gains dF)
    if (f >= 1) {
      const long long off = base + (long long)(s0 + f - 1) * st;
#pragma unroll
      for (int v = 0; v < NV; ++v) a.out[v * g.ncell + off] -= scale * (dF[v] * ph.inv_dx);
    }
    if (f < cnt) {
      const long long off = base + (long long)(s0 + f) * st;
#pragma unroll
      for (int v = 0; v < NV; ++v) a.out[v * g.ncell + off] += scale * (dF[v] * ph.inv_dx);
    }
  }
}

template <int NV, int DIR, int S, int OUT>
__global__ __launch_bounds__(SWEEP_BLOCK) void sweep_kernel(SweepArgs a, KGrid g, KPhys ph,
                                                            int nseg, long long nthreads) {
  const long long gid = (long long)blockIdx.x * SWEEP_BLOCK + threadIdx.x;
  if (gid >= nthreads) return;
  sweep_body<NV, DIR, S, OUT>(a, g, ph, nseg, gid);
}

}  // namespace wl2
