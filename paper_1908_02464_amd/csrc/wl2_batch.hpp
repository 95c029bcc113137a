// Batched form: many independent 1D/2D grids advanced by persistent kernels
// walking ragged work tables (one table per sweep phase), so a fixed launch
// shape serves any mix of grid sizes and the per-step launch sequence can be
// captured once in a hipGraph.  Every grid runs exactly the per-segment code
// of the single-grid path (sweep_body), with its own dt, clock and status, so
// its result is bit-identical to running it alone.
#pragma once
#include "wl2_kernels.hpp"

namespace wl2 {

// Device-resident descriptor of one admitted grid (one slot).
struct BGrid {
  KGrid g;
  KPhys ph;
  double* U;    // state U^n, updated in place by the third stage
  double* U1;   // stage buffers
  double* U2;
  double* acc;  // 2D: x-sweep partial sum
  StepCtl* ctl;
  double cfl_dx;
  int dim, nv;
  int nseg[2];        // segments per line along x and y
  long long nthr[2];  // threads of the x and y sweeps
  int active;
  int pad;
};

constexpr int BATCH_SEG_DEFAULT = 8;
constexpr int BATCH_MAX_SLOTS = 4096;
constexpr int BATCH_CHUNK = 4096;  // cells per reduction chunk

// Ragged table of one phase: entry k covers global work items
// [start[k], start[k+1]) of slot slot[k]; starts are multiples of 64 so that
// a wavefront never mixes two grids.
struct BTable {
  int n;
  int pad;
  long long total;
  int slot[BATCH_MAX_SLOTS];
  long long start[BATCH_MAX_SLOTS + 1];
};

// Reduction chunks: chunk c covers cells [first[c], first[c] + count[c]) of
// slot cslot[c].
struct BChunks {
  int n;
  int pad;
  int* cslot;
  long long* first;
  int* count;
};

__device__ __forceinline__ int table_find(const BTable* t, long long i) {
  int lo = 0, hi = t->n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t->start[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// PH = 0: x sweeps of all grids (1D: with the RK combination; 2D: into acc);
// PH = 1: y sweeps of the 2D grids (with the RK combination).  SEG cells per
// thread along the sweep (BGrid::nseg was computed for the same SEG).
template <int PH, int SEG>
__global__ __launch_bounds__(SWEEP_BLOCK) void batch_sweep_kernel(const BGrid* __restrict__ grids,
                                                                  const BTable* __restrict__ tab,
                                                                  int stage) {
  const long long total = tab->total;
  for (long long i = (long long)blockIdx.x * SWEEP_BLOCK + threadIdx.x; i < total;
       i += (long long)gridDim.x * SWEEP_BLOCK) {
    const int k = table_find(tab, i);
    const BGrid& G = grids[tab->slot[k]];
    const long long gid = i - tab->start[k];
    if (gid >= G.nthr[PH]) continue;  // wavefront padding
    if (!(G.ctl->dt > 0.0)) continue;  // finished (or not started) run
    const double* Uk = stage == 0 ? G.U : (stage == 1 ? G.U1 : G.U2);
    double* out = stage == 0 ? G.U1 : (stage == 1 ? G.U2 : G.U);
    const double ra = stage == 0 ? 0.0 : (stage == 1 ? 0.75 : 1.0 / 3.0);
    const double rb = stage == 0 ? 1.0 : (stage == 1 ? 0.25 : 2.0 / 3.0);
    if (G.dim == 1) {
      if (PH == 0) {
        SweepArgs a{Uk, out, nullptr, G.U, G.ctl, ra, rb};
        sweep_body<3, 0, SEG, OUT_RK>(a, G.g, G.ph, G.nseg[0], gid);
      }
    } else {
      if (PH == 0) {
        SweepArgs a{Uk, G.acc, nullptr, nullptr, G.ctl, 0.0, 1.0};
        sweep_body<4, 0, SEG, OUT_WRITE>(a, G.g, G.ph, G.nseg[0], gid);
      } else {
        SweepArgs a{Uk, out, G.acc, G.U, G.ctl, ra, rb};
        sweep_body<4, 1, SEG, OUT_RK>(a, G.g, G.ph, G.nseg[1], gid);
      }
    }
  }
}

// Per-grid CFL maximum over reduction chunks; one atomic per chunk.  The
// per-cell arithmetic is the same as cfl_reduce_kernel (bit-identical dt).
__global__ __launch_bounds__(RED_BLOCK) void batch_cfl_kernel(const BGrid* __restrict__ grids,
                                                              BChunks ch, const int* nchunks) {
#pragma clang fp contract(off)
  __shared__ double sh[RED_BLOCK / 64];
  const int n = *nchunks;
  for (int c = blockIdx.x; c < n; c += gridDim.x) {
    const BGrid& G = grids[ch.cslot[c]];
    const long long c0 = ch.first[c];
    const int cnt = ch.count[c];
    const long long nc = G.g.ncell;
    const double* U = G.U;
    const double gamma = G.ph.gamma;
    double smax = 0.0;
    bool bad = false;
    for (int q = threadIdx.x; q < cnt; q += RED_BLOCK) {
      const long long cc = c0 + q;
      if (G.dim == 1) {
        const double m[1] = {U[nc + cc]};
        smax = nan_max(smax, cfl_speed<1>(U[cc], m, U[2 * nc + cc], gamma, bad));
      } else {
        const double m[2] = {U[nc + cc], U[2 * nc + cc]};
        smax = nan_max(smax, cfl_speed<2>(U[cc], m, U[3 * nc + cc], gamma, bad));
      }
    }
    const double bm = block_max(smax, sh);
    if (threadIdx.x == 0 && (bm > 0.0 || bm != bm))
      atomicMax(&G.ctl->smax_bits, (unsigned long long)__double_as_longlong(bm));
    if (bad) atomicOr(&G.ctl->status, 1u);
  }
}

// One thread per active slot: dt from its maximum, clipped to its own t_end
// (dt = 0 once finished or after a non-physical state).
[[maybe_unused]] static __global__ void batch_finalize_kernel(const BGrid* __restrict__ grids, const int* slots,
                                      const int* nslots) {
  const int n = *nslots;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const BGrid& G = grids[slots[i]];
    StepCtl* ctl = G.ctl;
    double dt = G.cfl_dx / __longlong_as_double((long long)ctl->smax_bits);
    const double t = ctl->t, te = ctl->t_end;
    if (!(t < te) || ctl->status != 0u || !(dt > 0.0)) {
      dt = 0.0;
    } else {
      if (t + dt > te) dt = te - t;
      ctl->t = t + dt;
      ctl->steps += 1u;
    }
    ctl->dt = dt;
    ctl->smax_bits = 0ull;
  }
}

// Snapshot of every active slot's clock and status for the host poll.
struct SlotState {
  double t, t_end;
  unsigned int status;
  int slot;
};

[[maybe_unused]] static __global__ void batch_gather_kernel(const BGrid* __restrict__ grids, const int* slots,
                                    const int* nslots, SlotState* out) {
  const int n = *nslots;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const StepCtl* ctl = grids[slots[i]].ctl;
    out[i].t = ctl->t;
    out[i].t_end = ctl->t_end;
    out[i].status = ctl->status;
    out[i].slot = slots[i];
  }
}

}  // namespace wl2
