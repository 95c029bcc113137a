// Batched form: many independent 1D/2D grids advanced by persistent kernels
// walking tables of work items (one table per dimension), so a fixed launch
// shape serves any mix of grid sizes and the per-step launch sequence can be
// captured once in a hipGraph.  A work item is the unit of the single-grid
// row kernel (63 columns x a chunk of rows of one grid, one wavefront) and
// runs exactly its code (row_item), with the grid's own dt, clock and
// status, so a run's result is bit-identical to running it alone.
#pragma once
#include "wl2_aux.hpp"
#include "wl2_row.hpp"
#include "wl2_row_launch.hpp"

namespace wl2 {

// Device-resident descriptor of one admitted grid (one slot).
struct BGrid {
  KGrid g;
  KPhys ph;
  double* U;   // state U^n, updated in place by the third stage
  double* U1;  // stage buffers
  double* U2;
  StepCtl* ctl;
  double cfl_dx;
  int dim, nv;
  int active;
  int pad;
};

constexpr int BATCH_MAX_SLOTS = 4096;
constexpr int BATCH_CHUNK = 4096;  // cells per reduction chunk

// Work item of the batched row kernel: columns x0 .. x0+62 and rows y0 .. y1-1
// of the grid in `slot`.
struct RowItem {
  int slot, x0, y0, y1;
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

// Stage `stage` of every item of one dimension (NV = 3: 1D runs, 4: 2D).
// Stage pointers and RK coefficients of a run.
struct StageRefs {
  const double* Uk;
  double* out;
  double ra, rb;
};

__device__ __forceinline__ StageRefs stage_refs(const BGrid& G, int stage) {
  StageRefs r;
  r.Uk = stage == 0 ? G.U : (stage == 1 ? G.U1 : G.U2);
  r.out = stage == 0 ? G.U1 : (stage == 1 ? G.U2 : G.U);
  r.ra = stage == 0 ? 0.0 : (stage == 1 ? 0.75 : 1.0 / 3.0);
  r.rb = stage == 0 ? 1.0 : (stage == 1 ? 0.25 : 2.0 / 3.0);
  return r;
}

template <int NV>
__global__ __launch_bounds__(RW, 2) void batch_row_kernel(const BGrid* __restrict__ grids,
                                                         const RowItem* __restrict__ items,
                                                         const int* n_items, int stage,
                                                         unsigned long long* list,
                                                         unsigned int* list_n) {
  __shared__ double buf[NV + 3][RB];
  __shared__ double ring[2][NV + 3][RW];
  const int n = *n_items;
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
    const RowItem it = items[k];
    const BGrid& G = grids[it.slot];
    const double dt = G.ctl->dt;
    if (!(dt > 0.0)) continue;  // finished (or not started) run
    const StageRefs sr = stage_refs(G, stage);
    const RowArgs a{sr.Uk, sr.out, G.U, G.ctl, sr.ra, sr.rb, list, list_n,
                    (unsigned long long)it.slot << 40, nullptr, nullptr};
    // (a batch admits no grid with state sides: their checks compiled out)
    if (G.ph.split == SPLIT_LLF && G.ph.hybrid == HYB_PER_FIELD)
      row_item<NV, OUT_RK, 0, 0, false>(a, G.g, G.ph, buf, ring, it.x0, it.y0, it.y1, dt);
    else
      row_item<NV, OUT_RK, -1, -1, false>(a, G.g, G.ph, buf, ring, it.x0, it.y0, it.y1, dt);
  }
}

// Nonlinear corrections of the cells listed in this stage by all runs
// (entries slot << 40 | element offset << 8 | face mask): FIX_GRP lanes per
// entry for a short list, a lane per entry for a long one (same bits).
__global__ __launch_bounds__(128) void batch_fix_kernel(const BGrid* __restrict__ grids,
                                                        const unsigned long long* __restrict__ list,
                                                        const unsigned int* list_n, int stage) {
  const unsigned int n = *list_n;
  const unsigned int threads = gridDim.x * blockDim.x;
  const unsigned int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const bool grouped = (unsigned long long)n * FIX_GRP <= FIX_GROUPED_LANES && n <= threads / FIX_GRP;
  const unsigned int step = grouped ? threads / FIX_GRP : threads;
  for (unsigned int i = grouped ? tid / FIX_GRP : tid; i < n; i += step) {
    const unsigned long long e = list[i];
    const BGrid& G = grids[(int)(e >> 40)];
    const double dt = G.ctl->dt;
    if (!(dt > 0.0)) continue;
    const StageRefs sr = stage_refs(G, stage);
    const long long off = (long long)((e >> 8) & 0xffffffffull);
    const unsigned cm = (unsigned)(e & 0xffu);
    const bool fast = G.ph.split == SPLIT_LLF && G.ph.hybrid == HYB_PER_FIELD;
    if (G.dim == 1) {
      double un[3];
      if (fast) row_fix_cell<3, 0, 0>(sr.Uk, sr.out, G.ctl, G.g, G.ph, off, cm, sr.rb * dt, grouped, un);
      else row_fix_cell<3, -1, -1>(sr.Uk, sr.out, G.ctl, G.g, G.ph, off, cm, sr.rb * dt, grouped, un);
    } else {
      double un[4];
      if (fast) row_fix_cell<4, 0, 0>(sr.Uk, sr.out, G.ctl, G.g, G.ph, off, cm, sr.rb * dt, grouped, un);
      else row_fix_cell<4, -1, -1>(sr.Uk, sr.out, G.ctl, G.g, G.ph, off, cm, sr.rb * dt, grouped, un);
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
    if (threadIdx.x == 0 && (bm > 0.0 || bm != bm)) cfl_fold(G.ctl, bm);
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
    double dt = G.cfl_dx / cfl_take(ctl);
    const double t = ctl->t, te = ctl->t_end;
    if (!(t < te) || ctl->status != 0u || !(dt > 0.0)) {
      dt = 0.0;
    } else {
      if (t + dt > te) dt = te - t;
      ctl->t = t + dt;
      ctl->steps += 1u;
    }
    ctl->dt = dt;
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
