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
  int fast;      // LLF splitting with the per-field switch (compile-time path)
  int nvar;      // 3 (1D) or 4 (2D)
  unsigned long long* list;  // correction list (ncell entries) and its length
  unsigned int* list_n;
  KGrid g;
  KPhys ph;
  hipStream_t stream;
};

// The three launches of one stage, in stream order: clear the correction
// list, the row kernel, the nonlinear corrections of the listed cells.
hipError_t row_reset(const RowLaunch& L);
hipError_t row_launch(const RowLaunch& L);
hipError_t row_fix(const RowLaunch& L);

}  // namespace wl2
