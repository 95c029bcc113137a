// Fused 1D/2D stage kernel (gfx950, FP64): both sweep directions, the flux
// difference of Eq.(19) and the SSP-RK3 stage combination in one pass over
// HBM, for one grid (row_kernel) or for many grids (the batched form).
//
// Work item: one wavefront owns RT = 63 consecutive columns of one grid and
// marches along y through a chunk of rows (1D: the single row).  Each lane
// keeps a six-cell window of light records (U, p, c, 1/sqrt(rho)) of its
// column, four in registers and the two oldest in an LDS ring, so the y face
// of every row is formed without another load.  The current row plus a
// three-cell x halo is staged in LDS; lane t computes the x face on the left
// of column t (64 faces for 63 cells) and the right face of a cell arrives
// from the next lane by a cross-lane shuffle, so every face flux is computed
// once and both neighbours use the same bits.  Faces whose detector asks for
// the nonlinear flux are only flagged in the march: their cells go to a
// correction list and a separate kernel adds the WENO-L2IS part (one thread
// per listed cell, so a discontinuity does not serialise the item that holds
// it).  Rows are read with coalesced loads; the next row of the window and of
// the halo is prefetched a row ahead, with the sign flip of mirror ghosts
// applied at use.
#pragma once
#include "wl2_lface.hpp"

namespace wl2 {

constexpr int RW = 64;      // lanes of a work item (one wavefront)
constexpr int RT = RW - 1;  // columns owned by an item: RW x faces
constexpr int RB = RW + 5;  // row buffer: cells x0-3 .. x0+RW+1

struct RowArgs {
  const double* Uk;    // stage input
  double* out;         // RK: U^(k+1); WRITE: dU/dt
  const double* Un;    // RK: U^n (read when rk_a != 0)
  const StepCtl* ctl;  // dt and the global LF speeds
  double rk_a, rk_b;   // RK: out = rk_a U^n + rk_b (Uk + dt dU)
  unsigned long long* list;  // cells next to a face that needs the WENO flux
  unsigned int* list_n;      // entries in list
  unsigned long long tag;    // or-ed into every entry (the batch slot << 40)
  unsigned int* list_clear;  // if set: the next stage's counter, zeroed by the
                             // correction kernel
  StepCtl* cfl;              // RK: if set, fold the CFL speed of the new state
                             // into cfl->smax / status (next step's dt)
  StepCtl* clock;            // RK stage 1 of a step whose CFL maximum the step
                             // before folded: the stage kernel forms the step's
                             // dt itself (clock_dt_wave, with cfl_dx and the
                             // inflow speed floor s_floor) and its correction
                             // kernel commits the clock (clock_commit); else null
  double cfl_dx, s_floor;
};

// Entry of the correction list: tag | element offset << 8 | face mask (bit 0
// x-, 1 x+, 2 y-, 3 y+).  Appended with one atomic per wavefront.
__device__ __forceinline__ void list_append(const RowArgs& a, long long off, unsigned cm) {
  const unsigned long long ball = __ballot(cm != 0u);
  if (!ball) return;
  const int lane = threadIdx.x & (RW - 1);
  const int leader = __ffsll((long long)ball) - 1;
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(a.list_n, (unsigned int)__popcll(ball));
  base = __shfl(base, leader, RW);
  if (cm) {
    const unsigned int rank = __popcll(ball & ((1ull << lane) - 1ull));
    a.list[base + rank] = a.tag | ((unsigned long long)off << 8) | cm;
  }
}

template <int NV>
__device__ __forceinline__ void row_put(double (*buf)[RB], int i, const LRec<NV>& r) {
#pragma unroll
  for (int v = 0; v < NV; ++v) buf[v][i] = r.U[v];
  buf[NV][i] = r.p;
  buf[NV + 1][i] = r.c;
  buf[NV + 2][i] = r.iw;
}

template <int NV>
struct RowSrc {  // six cells of the row buffer from `base`
  double (*buf)[RB];
  int base;
  __device__ __forceinline__ void get(int m, LRec<NV>& r) const {
    const int i = base + m;
#pragma unroll
    for (int v = 0; v < NV; ++v) r.U[v] = buf[v][i];
    r.p = buf[NV][i];
    r.c = buf[NV + 1][i];
    r.iw = buf[NV + 2][i];
  }
};

// Per-lane ring of the two oldest cells of the y window: [2][NV+3][RW].
template <int NV>
__device__ __forceinline__ void ring_put(double (*ring)[NV + 3][RW], int slot, int lane,
                                         const LRec<NV>& r) {
#pragma unroll
  for (int v = 0; v < NV; ++v) ring[slot][v][lane] = r.U[v];
  ring[slot][NV][lane] = r.p;
  ring[slot][NV + 1][lane] = r.c;
  ring[slot][NV + 2][lane] = r.iw;
}

template <int NV>
struct RingSrc {  // y stencil: cells j-2, j-1 from the ring, j .. j+3 registers
  double (*ring)[NV + 3][RW];
  int slot0, slot1, lane;
  const LRec<NV>&r0, &r1, &r2, &r3;
  __device__ __forceinline__ void ring_get(int slot, LRec<NV>& r) const {
#pragma unroll
    for (int v = 0; v < NV; ++v) r.U[v] = ring[slot][v][lane];
    r.p = ring[slot][NV][lane];
    r.c = ring[slot][NV + 1][lane];
    r.iw = ring[slot][NV + 2][lane];
  }
  __device__ __forceinline__ void get(int m, LRec<NV>& r) const {
    if (m == 0) ring_get(slot0, r);
    else if (m == 1) ring_get(slot1, r);
    else r = m == 2 ? r0 : m == 3 ? r1 : m == 4 ? r2 : r3;
  }
};

template <int NV>
struct Win6Src {  // six records in registers
  const LRec<NV> (&w)[6];
  __device__ __forceinline__ void get(int m, LRec<NV>& r) const { r = w[m]; }
};

// Raw cell (column element offset xy, row y) of a 2D grid, ghost-mapped in
// y; the mirror flip of the y momentum is reported, not applied.
template <int NV, bool YS = true>
__device__ __forceinline__ void row_load_raw(const double* __restrict__ U, const KGrid& g,
                                             long long xy, int y, double (&u)[NV]) {
  bool fy = false;
  const int iy = (y >= 0 && y < g.n[1]) ? y : ghost_clamped(y, g.n[1], g.bc_lo[1], g.bc_hi[1], fy);
  const long long off = xy + (long long)iy * g.stride[1];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = U[v * g.ncell + off];
  // state ghosts of a y side (2D grids: xy is the column's x; YS false: the
  // caller's grids have none, and the check is compiled out)
  if (YS && NV == 4 && (y < 0 || y >= g.n[1]) && is_yghost(g, y)) load_yghost<NV>(g, xy, y, u);
}

template <int NV>
__device__ __forceinline__ void row_flip(const KGrid& g, bool fx, int y, double (&u)[NV]) {
  bool fy = false;
  if (NV >= 4 && (y < 0 || y >= g.n[1])) (void)ghost_clamped(y, g.n[1], g.bc_lo[1], g.bc_hi[1], fy);
  if (fx) u[1] = -u[1];
  if (NV >= 4 && fy) u[2] = -u[2];
}

// One work item: columns x0 .. x0+RT-1 (clipped to the grid), rows y0 .. y1-1
// (1D: y0 = 0, y1 = 1): the linear-branch fluxes of all its faces, Eq.(19)
// and the stage combination; cells next to a flagged face are listed.
// Called by whole wavefronts; `buf` is the item's LDS row buffer [NV+3][RB],
// `ring` its window ring [2][NV+3][RW] (2D).
template <int NV, int OUT, int SPLIT, int HYB, bool YS = true>
__device__ __forceinline__ void row_item(const RowArgs& a, const KGrid& g, const KPhys& ph,
                                         double (*buf)[RB], double (*ring)[NV + 3][RW], int x0,
                                         int y0, int y1, double dt) {
  const int lane = threadIdx.x & (RW - 1);
  const unsigned long long* lfx = a.ctl->lf_bits[0];
  const unsigned long long* lfy = a.ctl->lf_bits[1];
  // the lane's column (a ghost or the next item's column for lane RT and past
  // the grid edge: those fill the row buffer but own no cell)
  bool fx;
  const int cx = ghost_clamped(x0 + lane, g.n[0], g.bc_lo[0], g.bc_hi[0], fx);
  const bool own = lane < RT && x0 + lane < g.n[0];
  // halo cells: lanes 0-2 fill slots 0-2 (x0-3 .. x0-1), lanes 3-4 slots
  // RW+3, RW+4 (x0+RW, x0+RW+1)
  const bool halo = lane < 5;
  const int hslot = lane < 3 ? lane : RW + lane;
  bool fxh = false;
  const int hx = halo ? ghost_clamped(x0 - 3 + hslot, g.n[0], g.bc_lo[0], g.bc_hi[0], fxh) : 0;
  // halo ghost of an inflow side: its state comes from g.inflow
  const bool hin = halo && x0 - 3 + hslot < 0 && g.bc_lo[0] == BC_INFLOW;
  const long long oxy = cx;  // row 0 element offset of the column (x stride 1)
  const long long hxy = hx;
  double cfl_max = 0.0;  // CFL speed of the cells written here (a.cfl set)
  bool cfl_bad = false;

  if constexpr (NV == 3) {
    // 1D: one row
    double u[NV];
    row_load_raw<NV, YS>(a.Uk, g, oxy, 0, u);
    row_flip<NV>(g, fx, 0, u);
    LRec<NV> own_rec;
    make_lrec<NV>(u, ph, own_rec);
    row_put<NV>(buf, lane + 3, own_rec);
    if (halo) {
      double hu[NV];
      row_load_raw<NV, YS>(a.Uk, g, hxy, 0, hu);
      row_flip<NV>(g, fxh, 0, hu);
      if (hin) load_inflow<NV>(g, 0, hu);
      LRec<NV> hr;
      make_lrec<NV>(hu, ph, hr);
      row_put<NV>(buf, hslot, hr);
    }
    double unp[NV] = {};
    if (OUT == OUT_RK && a.rk_a != 0.0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) unp[v] = __builtin_nontemporal_load(&a.Un[v * g.ncell + oxy]);
    }
    __syncthreads();
    double Fx[NV];
    const unsigned mx =
        face_linear_l<NV, 0, SPLIT, HYB>(RowSrc<NV>{buf, lane}, ph, ph.eps_thr[0], lfx, Fx);
    double Fr[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fr[v] = __shfl_down(Fx[v], 1, RW);
    const unsigned mxr = __shfl_down(mx, 1, RW);
    const unsigned cm = own ? ((mx ? 1u : 0u) | (mxr ? 2u : 0u)) : 0u;
    list_append(a, oxy, cm);
    if (own) {
      double un[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double dU = (Fx[v] - Fr[v]) * ph.inv_dx;
        if (OUT == OUT_RK) {
          double r = a.rk_b * (own_rec.U[v] + dt * dU);
          if (a.rk_a != 0.0) r += a.rk_a * unp[v];
          __builtin_nontemporal_store(r, &a.out[v * g.ncell + oxy]);
          un[v] = r;
        } else {
          __builtin_nontemporal_store(dU, &a.out[v * g.ncell + oxy]);
        }
      }
      // a listed cell is finished (and its CFL speed counted) by the
      // correction kernel
      if (OUT == OUT_RK && a.cfl != nullptr && cm == 0u)
        cfl_max = nan_max(cfl_max, cfl_speed_u<NV>(un, ph.gamma, cfl_bad));
    }
    __syncthreads();  // the buffer is reused by the next item
  } else {
    // 2D: column window = cells y-2, y-1 (LDS ring, slot = row & 1) and
    // y .. y+3 (registers r0..r3) at the top of row y
    LRec<NV> r0, r1, r2, r3;
    double Fyp[NV];
    double upre[NV], hpre[NV];
    bool yprev;  // face y - 1/2 needs the nonlinear flux
    {
      LRec<NV> cm3, cm2, cm1;
      double u[NV];
      row_load_raw<NV, YS>(a.Uk, g, oxy, y0 - 3, u);
      row_flip<NV>(g, fx, y0 - 3, u);
      make_lrec<NV>(u, ph, cm3);
      row_load_raw<NV, YS>(a.Uk, g, oxy, y0 - 2, u);
      row_flip<NV>(g, fx, y0 - 2, u);
      make_lrec<NV>(u, ph, cm2);
      row_load_raw<NV, YS>(a.Uk, g, oxy, y0 - 1, u);
      row_flip<NV>(g, fx, y0 - 1, u);
      make_lrec<NV>(u, ph, cm1);
      row_load_raw<NV, YS>(a.Uk, g, oxy, y0, u);
      row_flip<NV>(g, fx, y0, u);
      make_lrec<NV>(u, ph, r0);
      row_load_raw<NV, YS>(a.Uk, g, oxy, y0 + 1, u);
      row_flip<NV>(g, fx, y0 + 1, u);
      make_lrec<NV>(u, ph, r1);
      row_load_raw<NV, YS>(a.Uk, g, oxy, y0 + 2, u);
      row_flip<NV>(g, fx, y0 + 2, u);
      make_lrec<NV>(u, ph, r2);
      row_load_raw<NV, YS>(a.Uk, g, oxy, y0 + 3, u);
      row_flip<NV>(g, fx, y0 + 3, u);
      make_lrec<NV>(u, ph, r3);
      ring_put<NV>(ring, (y0 - 2) & 1, lane, cm2);
      ring_put<NV>(ring, (y0 - 1) & 1, lane, cm1);
      // face y0 - 1/2: cells y0-3 .. y0+2
      const LRec<NV> wp[6] = {cm3, cm2, cm1, r0, r1, r2};
      yprev = face_linear_l<NV, 1, SPLIT, HYB>(Win6Src<NV>{wp}, ph, ph.eps_thr[1], lfy, Fyp) != 0u;
      row_load_raw<NV, YS>(a.Uk, g, oxy, y0 + 4, upre);
      if (halo) row_load_raw<NV, YS>(a.Uk, g, hxy, y0, hpre);
    }
    for (int y = y0; y < y1; ++y) {
      row_put<NV>(buf, lane + 3, r0);  // cell (x, y)
      if (halo) {
        row_flip<NV>(g, fxh, y, hpre);
        if (hin) load_inflow<NV>(g, y, hpre);
        LRec<NV> hr;
        make_lrec<NV>(hpre, ph, hr);
        row_put<NV>(buf, hslot, hr);
        asm volatile("" ::: "memory");  // the prefetch below stays after this use
        row_load_raw<NV, YS>(a.Uk, g, hxy, y + 1, hpre);
      }
      __syncthreads();
      __builtin_amdgcn_s_setprio(0);
      // x face on the left of column x0+lane (cells x-3 .. x+2 = slots lane .. lane+5)
      double Fx[NV];
      const unsigned mx =
          face_linear_l<NV, 0, SPLIT, HYB>(RowSrc<NV>{buf, lane}, ph, ph.eps_thr[0], lfx, Fx);
      const long long off = oxy + (long long)y * g.stride[1];
      double unp[NV] = {};
      if (OUT == OUT_RK && a.rk_a != 0.0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) unp[v] = __builtin_nontemporal_load(&a.Un[v * g.ncell + off]);
      }
      // y face y + 1/2: cells y-2, y-1 (ring), y .. y+3 (registers)
      double Fy[NV];
      const bool ycur = face_linear_l<NV, 1, SPLIT, HYB>(
                            RingSrc<NV>{ring, (y - 2) & 1, (y - 1) & 1, lane, r0, r1, r2, r3}, ph,
                            ph.eps_thr[1], lfy, Fy) != 0u;
      double Fr[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Fr[v] = __shfl_down(Fx[v], 1, RW);
      const unsigned mxr = __shfl_down(mx, 1, RW);
      const unsigned cm =
          own ? ((mx ? 1u : 0u) | (mxr ? 2u : 0u) | (yprev ? 4u : 0u) | (ycur ? 8u : 0u)) : 0u;
      list_append(a, off, cm);
      yprev = ycur;
      // raised wave priority from the stores through the next row's loads and
      // records to its barrier, normal for the faces (measured 1.6 % faster
      // on 2D 1024^2; local to this kernel)
      __builtin_amdgcn_s_setprio(2);
      if (own) {
        double un[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double dU = ((Fx[v] - Fr[v]) + (Fyp[v] - Fy[v])) * ph.inv_dx;
          if (OUT == OUT_RK) {
            double r = a.rk_b * (r0.U[v] + dt * dU);
            if (a.rk_a != 0.0) r += a.rk_a * unp[v];
            __builtin_nontemporal_store(r, &a.out[v * g.ncell + off]);
            un[v] = r;
          } else {
            __builtin_nontemporal_store(dU, &a.out[v * g.ncell + off]);
          }
        }
        if (OUT == OUT_RK && a.cfl != nullptr && cm == 0u)
          cfl_max = nan_max(cfl_max, cfl_speed_u<NV>(un, ph.gamma, cfl_bad));
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Fyp[v] = Fy[v];
      // retire cell y into the ring (over cell y-2), shift, make cell y+4
      // from the prefetch and prefetch y+5 into the freed registers
      ring_put<NV>(ring, y & 1, lane, r0);
      r0 = r1;
      r1 = r2;
      r2 = r3;
      row_flip<NV>(g, fx, y + 4, upre);
      make_lrec<NV>(upre, ph, r3);
      asm volatile("" ::"v"(r3.U[0]), "v"(r3.U[NV - 1]), "v"(r3.p), "v"(r3.c), "v"(r3.iw)
                   : "memory");
      row_load_raw<NV, YS>(a.Uk, g, oxy, y + 5, upre);
      __syncthreads();  // row buffer free for the next row
    }
  }
  if (OUT == OUT_RK && a.cfl != nullptr) cfl_commit_wave(a.cfl, cfl_max, cfl_bad);
}

// Lanes per listed cell in the correction kernels for short lists (one per
// face).
constexpr int FIX_GRP = 4;

// Nonlinear part of the flux of the flagged faces of one listed cell at
// element offset `off` (face order x-, x+, y-, y+, as in the 3D correction
// kernel), added to the output; `scale` = rk_b dt for a stage, 1 for dU/dt.
// grouped: FIX_GRP lanes share the cell (one face each) and the group's first
// lane writes; else one lane does all.  Each face is recomputed from the
// stage input by both of its cells with the same operations, so both get
// the same bits.  Returns true on the lane that wrote, with the new state in
// un.
template <int NV, int SPLIT, int HYB>
__device__ __forceinline__ bool row_fix_cell(const double* Uk, double* out, const StepCtl* ctl,
                                             const KGrid& g, const KPhys& ph, long long off,
                                             unsigned cm, double scale, bool grouped,
                                             double (&un)[NV]) {
  const int x = (int)(off % g.n[0]);
  const int y = (int)(off / g.n[0]);
  double acc[NV];
  if (grouped) grouped_correction<NV, FIX_GRP, SPLIT, HYB>(Uk, g, ph, ctl, x, y, 0, cm, acc);
  else serial_correction<NV, SPLIT, HYB>(Uk, g, ph, ctl, x, y, 0, cm, acc);
  if (grouped && (threadIdx.x % FIX_GRP) != 0) return false;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    un[v] = out[v * g.ncell + off] + scale * (acc[v] * ph.inv_dx);
    out[v * g.ncell + off] = un[v];
  }
  return true;
}

// Listed cells per workgroup round of the field-parallel mode: the two
// wavefronts of a 2D workgroup take the x and the y faces of 8 cells, one
// lane per (side, field) pair (8 of them); in 1D each takes 8 cells' x faces
// (6 lanes each).
template <int NV>
constexpr int fix_fields_cells() { return NV == 4 ? 8 : 16; }

// Field-parallel corrections of a short list (every cell in flight at once):
// each flagged face's change is formed by NV lanes, one per field
// (face_delta_field), a wavefront running one direction only, so a lane's
// work is the linear face and one field's WENO flux where one lane per face
// runs every flagged field and both directions one after the other.  The
// changes meet in LDS and are summed per cell in the fixed order x-, x+, y-,
// y+ as serial_correction sums them: the same bits.
template <int NV, int OUT, int SPLIT, int HYB>
__device__ __forceinline__ void row_fix_fields(const RowArgs& a, const KGrid& g, const KPhys& ph,
                                               unsigned int n, double scale, double& cfl_max,
                                               bool& cfl_bad) {
  constexpr int NF = 2 * (NV - 2);
  constexpr int CPB = fix_fields_cells<NV>();
  __shared__ double sdf[CPB][NF][NV];
  const int lane = threadIdx.x & 63;
  const int dir = NV == 4 ? (int)(threadIdx.x >> 6) : 0;
  const int cslot = NV == 4 ? (lane >> 3) : (int)(threadIdx.x >> 3);
  const int j = lane & 7, side = j / NV, k = j % NV;
  const int f = 2 * dir + side;
  const bool worker = j < 2 * NV;
  for (unsigned int base = blockIdx.x * CPB; base < n; base += gridDim.x * CPB) {
    const unsigned int i = base + cslot;
    unsigned cm = 0;
    long long off = 0;
    if (i < n) {
      const unsigned long long e = a.list[i];
      off = (long long)((e >> 8) & 0xffffffffull);
      cm = (unsigned)(e & 0xffu);
    }
    double dF[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) dF[v] = 0.0;
    if (worker && ((cm >> f) & 1u)) {
      const int x = (int)(off % g.n[0]), y = (int)(off / g.n[0]);
      const int lane0 = (lane & ~7) + side * NV;
      if (dir == 0) {
        face_delta_field<NV, 0, SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[0], x, y, 0, side, k, lane0, dF);
      } else {
        if constexpr (NV >= 4)
          face_delta_field<NV, 1, SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[1], x, y, 0, side, k, lane0, dF);
      }
    }
    if (worker && k == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sdf[cslot][f][v] = dF[v];
    }
    __syncthreads();
    if (threadIdx.x < CPB && base + threadIdx.x < n) {
      const unsigned long long e = a.list[base + threadIdx.x];
      const long long c = (long long)((e >> 8) & 0xffffffffull);
      const unsigned m = (unsigned)(e & 0xffu);
      double acc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
      for (int ff = 0; ff < NF; ++ff) {
        if (!((m >> ff) & 1u)) continue;
        const double sg = (ff & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += sg * sdf[threadIdx.x][ff][v];
      }
      double un[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        un[v] = a.out[v * g.ncell + c] + scale * (acc[v] * ph.inv_dx);
        a.out[v * g.ncell + c] = un[v];
      }
      if (OUT == OUT_RK && a.cfl != nullptr) cfl_max = nan_max(cfl_max, cfl_speed_u<NV>(un, ph.gamma, cfl_bad));
    }
    __syncthreads();  // sdf is free for the next round
  }
}

// Single grid.  A list short enough for every cell to be in flight at once
// (launched with 2048 workgroups: 16384 cells in 2D, 32768 in 1D) takes the
// field-parallel mode (latency), a longer one a lane per cell (throughput).
// 128 threads per workgroup.
template <int NV, int OUT, int SPLIT, int HYB>
__global__ __launch_bounds__(128) void row_fix_kernel(RowArgs a, KGrid g, KPhys ph) {
  // the next stage's list starts empty (no kernel of this stage uses it)
  if (a.list_clear != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.list_clear = 0u;
  if (a.clock != nullptr && blockIdx.x == 0 && threadIdx.x == 0) clock_commit(a.clock);
  double scale = 1.0;
  if (OUT == OUT_RK) {
    const double dt = a.ctl->dt;
    if (!(dt > 0.0)) return;
    scale = a.rk_b * dt;
  }
  const unsigned int n = *a.list_n;
  const unsigned int threads = gridDim.x * blockDim.x;
  const unsigned int tid = blockIdx.x * blockDim.x + threadIdx.x;
  double cfl_max = 0.0;
  bool cfl_bad = false;
  if ((unsigned long long)n <= (unsigned long long)gridDim.x * fix_fields_cells<NV>()) {
    row_fix_fields<NV, OUT, SPLIT, HYB>(a, g, ph, n, scale, cfl_max, cfl_bad);
  } else {
    for (unsigned int i = tid; i < n; i += threads) {
      const unsigned long long e = a.list[i];
      double un[NV];
      const bool wrote = row_fix_cell<NV, SPLIT, HYB>(a.Uk, a.out, a.ctl, g, ph,
                                                      (long long)((e >> 8) & 0xffffffffull),
                                                      (unsigned)(e & 0xffu), scale, false, un);
      if (OUT == OUT_RK && a.cfl != nullptr && wrote)
        cfl_max = nan_max(cfl_max, cfl_speed_u<NV>(un, ph.gamma, cfl_bad));
    }
  }
  if (OUT == OUT_RK && a.cfl != nullptr) cfl_commit_wave(a.cfl, cfl_max, cfl_bad);
}

// Face-once corrections of a long list (single grid).  Every flagged face
// is shared by two listed cells; the per-cell kernel above computes it for
// each of them.  Here phase A computes, per listed cell, the flagged face
// below it in each direction (x-, y-) once, into D[dir][v][entry], and
// records the cell's entry index in map; phase B sums, per listed cell, its
// flagged faces in the order x-, x+, y-, y+, taking a face above the cell
// from the entry of the cell above it (listed, since the face is flagged)
// or, where that cell is a ghost, computing it.  A face's change of flux has
// the same bits whichever cell computes it, and the sum is the per-cell
// kernel's, so the result is bit-identical.  A list short enough for all of
// its faces' fields to be in flight at once takes phase A field-parallel.
template <int NV, int OUT, int SPLIT, int HYB>
__global__ __launch_bounds__(128) void row_face_kernel(RowArgs a, KGrid g, KPhys ph, double* D,
                                                       unsigned int* map, unsigned int cap) {
  // the next stage's list starts empty (no kernel of this stage uses it)
  if (a.list_clear != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.list_clear = 0u;
  if (a.clock != nullptr && blockIdx.x == 0 && threadIdx.x == 0) clock_commit(a.clock);
  if (OUT == OUT_RK && !(a.ctl->dt > 0.0)) return;
  constexpr int ND = NV - 2;
  const unsigned int n = *a.list_n;
  const unsigned int threads = gridDim.x * blockDim.x;
  if ((unsigned long long)ND * n * NV <= threads) {
    // a short list: NV lanes per face, one per field (face_delta_field),
    // every face in flight at once; groups of NV consecutive lanes
    // (direction-major, then entry), so a group never straddles wavefronts
    const unsigned int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ND * n * NV) return;
    const unsigned int q = i / NV, kf = i - q * NV;
    const unsigned int dir = q / n, k = q - dir * n;
    const unsigned long long e = a.list[k];
    const long long off = (long long)((e >> 8) & 0xffffffffull);
    const unsigned cm = (unsigned)(e & 0xffu);
    if (dir == 0 && kf == 0) map[off] = k;
    if (!((cm >> (2 * dir)) & 1u)) return;
    const int x = (int)(off % g.n[0]);
    const int y = (int)(off / g.n[0]);
    const int lane0 = (int)(threadIdx.x & 63) - (int)kf;
    double dF[NV];
    if (dir == 0) {
      face_delta_field<NV, 0, SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[0], x, y, 0, 0, (int)kf, lane0, dF);
    } else {
      if constexpr (NV >= 4)
        face_delta_field<NV, (NV >= 4 ? 1 : 0), SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[1], x, y, 0, 0,
                                                            (int)kf, lane0, dF);
    }
    double val = dF[0];
#pragma unroll
    for (int v = 1; v < NV; ++v) val = v == (int)kf ? dF[v] : val;
    D[((size_t)dir * NV + kf) * cap + k] = val;  // lane kf writes value kf
    return;
  }
  // lanes ordered direction-major, so a wavefront takes faces of one direction
  for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < ND * n; i += threads) {
    const unsigned int dir = i / n, k = i - dir * n;
    const unsigned long long e = a.list[k];
    const long long off = (long long)((e >> 8) & 0xffffffffull);
    const unsigned cm = (unsigned)(e & 0xffu);
    if (dir == 0) map[off] = k;
    if (!((cm >> (2 * dir)) & 1u)) continue;
    const int x = (int)(off % g.n[0]);
    const int y = (int)(off / g.n[0]);
    double dF[NV];
    if (dir == 0) {
      face_delta<NV, 0, SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[0], x, y, 0, 0, dF);
    } else {
      if constexpr (NV >= 4)
        face_delta<NV, (NV >= 4 ? 1 : 0), SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[1], x, y, 0, 0, dF);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) D[((size_t)dir * NV + v) * cap + k] = dF[v];
  }
}

template <int NV, int OUT, int SPLIT, int HYB>
__global__ __launch_bounds__(128) void row_sum_kernel(RowArgs a, KGrid g, KPhys ph,
                                                      const double* __restrict__ D,
                                                      const unsigned int* __restrict__ map,
                                                      unsigned int cap) {
  double scale = 1.0;
  if (OUT == OUT_RK) {
    const double dt = a.ctl->dt;
    if (!(dt > 0.0)) return;
    scale = a.rk_b * dt;
  }
  constexpr int ND = NV - 2;
  const unsigned int n = *a.list_n;
  const unsigned int threads = gridDim.x * blockDim.x;
  double cfl_max = 0.0;
  bool cfl_bad = false;
  for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += threads) {
    const unsigned long long e = a.list[k];
    const long long off = (long long)((e >> 8) & 0xffffffffull);
    const unsigned cm = (unsigned)(e & 0xffu);
    const int x = (int)(off % g.n[0]);
    const int y = (int)(off / g.n[0]);
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
    for (int f = 0; f < 2 * ND; ++f) {
      if (!((cm >> f) & 1u)) continue;
      const int dir = f >> 1, side = f & 1;
      double d[NV];
      if (side == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) d[v] = D[((size_t)dir * NV + v) * cap + k];
      } else {
        const int pos = dir == 0 ? x : y;
        if (pos + 1 < g.n[dir]) {
          // the cell above is listed in this stage (its face below is the
          // flagged face); min() only keeps a broken list inside D
          const unsigned int kk = min(map[off + (dir == 0 ? 1ll : g.stride[1])], cap - 1u);
#pragma unroll
          for (int v = 0; v < NV; ++v) d[v] = D[((size_t)dir * NV + v) * cap + kk];
        } else if (dir == 0) {
          face_delta<NV, 0, SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[0], x, y, 0, 1, d);
        } else {
          if constexpr (NV >= 4)
            face_delta<NV, (NV >= 4 ? 1 : 0), SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[1], x, y, 0, 1, d);
        }
      }
      const double sg = side ? -1.0 : 1.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += sg * d[v];
    }
    double un[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      un[v] = a.out[v * g.ncell + off] + scale * (acc[v] * ph.inv_dx);
      a.out[v * g.ncell + off] = un[v];
    }
    if (OUT == OUT_RK && a.cfl != nullptr)
      cfl_max = nan_max(cfl_max, cfl_speed_u<NV>(un, ph.gamma, cfl_bad));
  }
  if (OUT == OUT_RK && a.cfl != nullptr) cfl_commit_wave(a.cfl, cfl_max, cfl_bad);
}

// Small 1D grids: whole SSP-RK3 steps in one workgroup of W wavefronts and
// one launch (the launches of the stage kernels, not their work, bound such
// grids).  Per step: the CFL maximum of U (cfl_speed, an exact maximum),
// the clock rule of finalize_dt_kernel, then per stage the row items (item
// k on wavefront k mod W, every wavefront taking the same number of items,
// past the grid edge owning no cell) and the corrections of the listed
// cells (field-parallel for up to nthr / 16 cells), with workgroup
// barriers between.  The same row_item, face_delta_field and row_fix_cell
// code as the multi-launch path: the same bits.
struct RowStepsArgs {
  double* U;             // state, advanced in place
  double* U1;            // stage states
  double* U2;
  StepCtl* ctl;          // clock, t_end, status, dt
  unsigned long long* list;
  double cfl_dx;         // CFL number x dx
  int n_steps;
};

template <int W, int SPLIT, int HYB>
__global__ __launch_bounds__(W * RW) void row1d_steps_kernel(RowStepsArgs s, KGrid g, KPhys ph) {
  constexpr int NV = 3;
  __shared__ double buf[W][NV + 3][RB];
  __shared__ double red[W];
  __shared__ unsigned int flags;  // bit 0: a non-physical cell in U
  __shared__ unsigned int list_n;
  __shared__ double s_dt;
  const int wave = threadIdx.x / RW, lane = threadIdx.x % RW;
  const int nthr = W * RW;
  const int n = g.n[0];
  const int per_wave = ((n + RT - 1) / RT + W - 1) / W;
  StepCtl* ctl = s.ctl;
  for (int step = 0; step < s.n_steps; ++step) {
    double m = 0.0;
    bool bad = false;
    for (int c = threadIdx.x; c < n; c += nthr) {
      double u[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = s.U[v * g.ncell + c];
      m = nan_max(m, cfl_speed_u<NV>(u, ph.gamma, bad));
    }
    // a NaN maximum is raised to +inf so that it wins (as in every reduction)
    const double wm = wave_max(m != m ? __longlong_as_double(0x7ff0000000000000LL) : m);
    const unsigned long long anybad = __ballot(bad);
    if (threadIdx.x == 0) flags = 0u;
    if (lane == 0) red[wave] = wm;
    __syncthreads();
    if (lane == 0 && anybad) atomicOr(&flags, 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
      double smax = 0.0;
#pragma unroll
      for (int w = 0; w < W; ++w) smax = fmax(smax, red[w]);
      if (flags) ctl->status |= 1u;
      double dt = s.cfl_dx / smax;
      const double t = ctl->t, te = ctl->t_end;
      if (!(t < te) || ctl->status != 0u) {
        dt = 0.0;
      } else {
        if (t + dt > te) dt = te - t;
        ctl->t = t + dt;
        ctl->steps += 1u;
      }
      ctl->dt = dt;
      s_dt = dt;
    }
    __syncthreads();
    const double dt = s_dt;
    if (!(dt > 0.0)) break;  // the clock has stopped (uniform)
    for (int st = 0; st < 3; ++st) {
      const double* Uk = st == 0 ? s.U : (st == 1 ? s.U1 : s.U2);
      double* out = st == 0 ? s.U1 : (st == 1 ? s.U2 : s.U);
      const double ra = st == 0 ? 0.0 : (st == 1 ? 0.75 : 1.0 / 3.0);
      const double rb = st == 0 ? 1.0 : (st == 1 ? 0.25 : 2.0 / 3.0);
      if (threadIdx.x == 0) list_n = 0u;
      __syncthreads();
      const RowArgs a{Uk, out, s.U, ctl, ra, rb, s.list, &list_n, 0ull, nullptr, nullptr};
      for (int k = 0; k < per_wave; ++k)
        row_item<NV, OUT_RK, SPLIT, HYB>(a, g, ph, buf[wave], nullptr, (wave + k * W) * RT, 0, 1, dt);
      __syncthreads();
      const unsigned int nl = list_n;
      if (nl == 0u) {
        // nothing listed
      } else if ((unsigned long long)nl * 8u <= (unsigned long long)nthr / 2u) {
        // a list this short leaves the workgroup's SIMDs mostly idle:
        // field-parallel, 8 lanes per listed cell (one wavefront holds the
        // group), lane (side, field) of the first six forming that field's
        // change of the face below (side 0) or above (side 1) the cell; the
        // group's first lane sums the two faces as serial_correction does.
        // (Longer lists: the redundant linear faces of the field lanes cost
        // more than the shorter chains save on one CU.)
        const unsigned int i = threadIdx.x / 8;
        const int j = threadIdx.x % 8, side = j / NV, k = j % NV;
        unsigned long long e = 0ull;
        if (i < nl) e = s.list[i];
        const long long off = (long long)((e >> 8) & 0xffffffffull);
        const unsigned cm = i < nl ? (unsigned)(e & 0xffu) : 0u;
        double dF[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) dF[v] = 0.0;
        if (j < 2 * NV && ((cm >> side) & 1u))
          face_delta_field<NV, 0, SPLIT, HYB>(Uk, g, ph, ctl->lf_bits[0], (int)off, 0, 0, side, k,
                                              (lane & ~7) + side * NV, dF);
        double dm[NV], dp[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          dm[v] = __shfl(dF[v], (lane & ~7), 64);
          dp[v] = __shfl(dF[v], (lane & ~7) + NV, 64);
        }
        if (i < nl && j == 0) {
          double acc[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[v] = 0.0;
          if (cm & 1u) {
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += 1.0 * dm[v];
          }
          if (cm & 2u) {
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += -1.0 * dp[v];
          }
#pragma unroll
          for (int v = 0; v < NV; ++v)
            out[v * g.ncell + off] = out[v * g.ncell + off] + (rb * dt) * (acc[v] * ph.inv_dx);
        }
      } else {
        const bool grouped = (unsigned long long)nl * FIX_GRP <= (unsigned long long)nthr;
        const unsigned int stride = grouped ? nthr / FIX_GRP : nthr;
        for (unsigned int i = grouped ? threadIdx.x / FIX_GRP : threadIdx.x; i < nl; i += stride) {
          const unsigned long long e = s.list[i];
          double un[NV];
          row_fix_cell<NV, SPLIT, HYB>(Uk, out, ctl, g, ph, (long long)((e >> 8) & 0xffffffffull),
                                       (unsigned)(e & 0xffu), rb * dt, grouped, un);
        }
      }
      __syncthreads();
    }
  }
}

[[maybe_unused]] static __global__ void row_list_reset_kernel(unsigned int* n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *n = 0u;
}

// Single grid: item = (x tile, chunk of `ych` rows), one wavefront each.
template <int NV, int OUT, int SPLIT, int HYB>
__global__ __launch_bounds__(RW, 2) void row_kernel(RowArgs a, KGrid g, KPhys ph, int ych,
                                                    int tiles_x) {
  __shared__ double buf[NV + 3][RB];
  __shared__ double ring[2][NV + 3][RW];
  double dt = 0.0;
  if (OUT == OUT_RK) {
    dt = a.clock != nullptr
             ? clock_dt_wave(a.clock, a.cfl_dx, a.s_floor, blockIdx.x == 0 && threadIdx.x == 0)
             : a.ctl->dt;
    if (!(dt > 0.0)) return;  // finished run: leave the state untouched
  }
  const int item = blockIdx.x;
  const int tx = item % tiles_x, ty = item / tiles_x;
  const int y0 = ty * ych;
  const int y1 = min(y0 + ych, g.n[1]);
  row_item<NV, OUT, SPLIT, HYB>(a, g, ph, buf, ring, tx * RT, y0, y1, dt);
}

}  // namespace wl2
