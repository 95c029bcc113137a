// Launch interface of the fused 1D/2D row kernels (wl2_row.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "wl2_device.hpp"

namespace wl2 {

constexpr int ROW_TILE = 63;     // columns per work item (one wavefront)
constexpr int ROW_MAX_YCH = 62;  // rows per work item (flag bits per row)

struct RowLaunch {
  const double* Uk;
  double* out;
  const double* Un;
  const StepCtl* ctl;
  double rk_a, rk_b;
  int out_kind;  // OUT_WRITE or OUT_RK
  int ych;       // rows per work item (2D)
  int fast;      // compile-time build with the per-field switch: 1 = LLF
                 // splitting, 2 = global LF splitting, 0 = the scheme read at
                 // run time
  int nvar;      // 3 (1D) or 4 (2D)
  unsigned long long* list;  // correction list (ncell entries) and its length
  unsigned int* list_n;
  unsigned int* list_clear;  // the next stage's counter, zeroed by the correction kernel
  StepCtl* cfl;              // RK: fold the CFL speed of the new state here (or null)
  StepCtl* clock;            // RK stage 1: the stage kernel forms the step's dt
                             // from the CFL maximum folded here (or null)
  double cfl_dx, s_floor;    // with clock: CFL number x dx, inflow speed floor
  // face-once corrections (2D, long lists): per-entry face changes
  // [2][nvar][fo_cap] and the cell -> entry map [ncell]; null: per cell
  double* fo_D;
  unsigned int* fo_map;
  unsigned int fo_cap;
  KGrid g;
  KPhys ph;
  hipStream_t stream;
};

// The launches of one stage, in stream order: the row kernel and the
// nonlinear corrections of the listed cells.  The list counter of a stage is
// cleared by the previous stage's correction kernel; row_reset clears both
// counters (before the first stage, or after a failed launch).
hipError_t row_reset(const RowLaunch& L);
hipError_t row_launch(const RowLaunch& L);
hipError_t row_fix(const RowLaunch& L);

// Small 1D grids: n_steps clock steps of U (SSP-RK3, device CFL dt, the
// clock rule of the multi-launch path) in one single-workgroup launch of
// eight wavefronts (measured per step against seven launches: 200 cells
// 19 vs 33 us, 800 cells 26 vs 34 us, 1024 cells 31 vs 33 us, 1600 cells
// 38 vs 35 us; sixteen wavefronts spill).
constexpr int ROW_STEPS_MAX_CELLS = 1024;
hipError_t row1d_steps(double* U, double* U1, double* U2, StepCtl* ctl, unsigned long long* list,
                       double cfl_dx, int n_steps, int fast, const KGrid& g, const KPhys& ph,
                       hipStream_t stream);

}  // namespace wl2
