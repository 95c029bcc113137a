// Dispatch of the fused 1D/2D row kernels (wl2_row.hpp).
#include <hip/hip_runtime.h>

#include "wl2_row.hpp"
#include "wl2_row_launch.hpp"

namespace wl2 {

static_assert(ROW_TILE == RT, "one tile width for host and device");

namespace {

// Builds: LLF or global-LF splitting with the per-field switch fixed at
// compile time (the paper's 1D and 2D choices), any other scheme read at
// run time (those builds spill; at 1024^2 global LF took 0.26 ms per step
// through them against 0.19 for the LLF build).
template <int NV, int OUT>
void launch_nv(const RowLaunch& L, const RowArgs& a, dim3 grid, int ych, int tiles_x) {
  if (L.fast == 1)
    hipLaunchKernelGGL((row_kernel<NV, OUT, SPLIT_LLF, HYB_PER_FIELD>), grid, dim3(RW), 0, L.stream, a, L.g, L.ph, ych, tiles_x);
  else if (L.fast == 2)
    hipLaunchKernelGGL((row_kernel<NV, OUT, SPLIT_LF, HYB_PER_FIELD>), grid, dim3(RW), 0, L.stream, a, L.g, L.ph, ych, tiles_x);
  else
    hipLaunchKernelGGL((row_kernel<NV, OUT, -1, -1>), grid, dim3(RW), 0, L.stream, a, L.g, L.ph, ych, tiles_x);
}

}  // namespace

hipError_t row_reset(const RowLaunch& L) {
  hipLaunchKernelGGL(row_list_reset_kernel, dim3(1), dim3(64), 0, L.stream, L.list_n);
  if (L.list_clear != nullptr)
    hipLaunchKernelGGL(row_list_reset_kernel, dim3(1), dim3(64), 0, L.stream, L.list_clear);
  return hipGetLastError();
}

hipError_t row1d_steps(double* U, double* U1, double* U2, StepCtl* ctl, unsigned long long* list,
                       double cfl_dx, int n_steps, int fast, const KGrid& g, const KPhys& ph,
                       hipStream_t stream) {
  constexpr int W = 8;
  if (g.n[1] != 1 || g.n[2] != 1 || g.n[0] > ROW_STEPS_MAX_CELLS) return hipErrorInvalidValue;
  const RowStepsArgs s{U, U1, U2, ctl, list, cfl_dx, n_steps};
  if (fast == 1)
    hipLaunchKernelGGL((row1d_steps_kernel<W, SPLIT_LLF, HYB_PER_FIELD>), dim3(1), dim3(W * RW), 0, stream, s, g, ph);
  else
    hipLaunchKernelGGL((row1d_steps_kernel<W, -1, -1>), dim3(1), dim3(W * RW), 0, stream, s, g, ph);
  return hipGetLastError();
}

hipError_t row_fix(const RowLaunch& L) {
  const RowArgs a{L.Uk,   L.out,    L.Un, L.ctl,        L.rk_a,
                  L.rk_b, L.list,   L.list_n, 0ull, L.list_clear,
                  L.out_kind == OUT_RK ? L.cfl : nullptr, L.out_kind == OUT_RK ? L.clock : nullptr,
                  L.cfl_dx, L.s_floor};
  const dim3 fg(1024), fb(128);
  // the per-cell kernel: 2048 workgroups, so that lists of up to 16384
  // cells take its field-parallel mode (workgroups past the list's end
  // return at once)
  const dim3 fgc(2048);
  if (L.fo_D != nullptr) {
    if (L.nvar != 4) return hipErrorInvalidValue;
#define WL2_FO(O, S, H)                                                                          \
  do {                                                                                           \
    hipLaunchKernelGGL((row_face_kernel<4, O, S, H>), fg, fb, 0, L.stream, a, L.g, L.ph, L.fo_D,  \
                       L.fo_map, L.fo_cap);                                                      \
    hipLaunchKernelGGL((row_sum_kernel<4, O, S, H>), fg, fb, 0, L.stream, a, L.g, L.ph, L.fo_D,   \
                       L.fo_map, L.fo_cap);                                                      \
  } while (0)
    if (L.out_kind == OUT_RK) {
      if (L.fast == 1) WL2_FO(OUT_RK, SPLIT_LLF, HYB_PER_FIELD);
      else if (L.fast == 2) WL2_FO(OUT_RK, SPLIT_LF, HYB_PER_FIELD);
      else WL2_FO(OUT_RK, -1, -1);
    } else {
      if (L.fast == 1) WL2_FO(OUT_WRITE, SPLIT_LLF, HYB_PER_FIELD);
      else if (L.fast == 2) WL2_FO(OUT_WRITE, SPLIT_LF, HYB_PER_FIELD);
      else WL2_FO(OUT_WRITE, -1, -1);
    }
#undef WL2_FO
    return hipGetLastError();
  }
#define WL2_FIX(NV, O)                                                                     \
  do {                                                                                     \
    if (L.fast == 1)                                                                       \
      hipLaunchKernelGGL((row_fix_kernel<NV, O, SPLIT_LLF, HYB_PER_FIELD>), fgc, fb, 0, L.stream, a, L.g, L.ph); \
    else if (L.fast == 2)                                                                  \
      hipLaunchKernelGGL((row_fix_kernel<NV, O, SPLIT_LF, HYB_PER_FIELD>), fgc, fb, 0, L.stream, a, L.g, L.ph); \
    else                                                                                   \
      hipLaunchKernelGGL((row_fix_kernel<NV, O, -1, -1>), fgc, fb, 0, L.stream, a, L.g, L.ph); \
  } while (0)
  if (L.nvar == 3) {
    if (L.out_kind == OUT_RK) WL2_FIX(3, OUT_RK); else WL2_FIX(3, OUT_WRITE);
  } else if (L.nvar == 4) {
    if (L.out_kind == OUT_RK) WL2_FIX(4, OUT_RK); else WL2_FIX(4, OUT_WRITE);
  } else {
    return hipErrorInvalidValue;
  }
#undef WL2_FIX
  return hipGetLastError();
}

hipError_t row_launch(const RowLaunch& L) {
  const RowArgs a{L.Uk,   L.out,  L.Un,     L.ctl, L.rk_a,
                  L.rk_b, L.list, L.list_n, 0ull,  nullptr,
                  L.out_kind == OUT_RK ? L.cfl : nullptr, L.out_kind == OUT_RK ? L.clock : nullptr,
                  L.cfl_dx, L.s_floor};
  const int tiles_x = (L.g.n[0] + RT - 1) / RT;
  const int ych = L.nvar == 3 ? 1 : (L.ych < 1 ? 1 : (L.ych > ROW_MAX_YCH ? ROW_MAX_YCH : L.ych));
  const long long chunks = L.nvar == 3 ? 1 : (L.g.n[1] + ych - 1) / ych;
  const long long items = (long long)tiles_x * chunks;
  if (items < 1 || items > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)items);
  if (L.nvar == 3) {
    if (L.out_kind == OUT_RK) launch_nv<3, OUT_RK>(L, a, grid, ych, tiles_x);
    else launch_nv<3, OUT_WRITE>(L, a, grid, ych, tiles_x);
  } else if (L.nvar == 4) {
    if (L.out_kind == OUT_RK) launch_nv<4, OUT_RK>(L, a, grid, ych, tiles_x);
    else launch_nv<4, OUT_WRITE>(L, a, grid, ych, tiles_x);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wl2
