// Dispatch of the fused 3D stage kernels (wl2_fused.hpp).
#include <hip/hip_runtime.h>

#include "wl2_fused.hpp"
#include "wl2_fused_launch.hpp"

namespace wl2 {

namespace {

FusedArgs make_args(const FusedLaunch& L) {
  FusedArgs a;
  a.Uk = L.Uk;
  a.out = L.out;
  a.Un = L.Un;
  a.ctl = L.ctl;
  a.rk_a = L.rk_a;
  a.rk_b = L.rk_b;
  a.zc = L.zc;
  a.list = L.list;
  a.list_n = L.list_n;
  a.list_clear = L.list_clear;
  a.cfl = L.out_kind == OUT_RK ? L.cfl : nullptr;
  a.tiles_x = (L.n[0] + FT_X - 1) / FT_X;
  a.tiles_y = (L.n[1] + FT_Y - 1) / FT_Y;
  return a;
}

}  // namespace

hipError_t fused3d_reset(const FusedLaunch& L) {
  hipLaunchKernelGGL(reset_list_kernel, dim3(1), dim3(64), 0, L.stream, L.list_n);
  hipLaunchKernelGGL(reset_list_kernel, dim3(1), dim3(64), 0, L.stream, L.list_clear);
  return hipGetLastError();
}

hipError_t fused3d_main(const FusedLaunch& L) {
  const FusedArgs a = make_args(L);
  const long long nzc = (L.n[2] + a.zc - 1) / a.zc;
  const long long blocks = (long long)a.tiles_x * a.tiles_y * nzc;
  if (a.zc < 1 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 gr((unsigned)blocks), bl(FT_THREADS);
#define WL2_FUSED(O, W, S, H) \
  hipLaunchKernelGGL((fused3d_kernel<O, W, S, H>), gr, bl, 0, L.stream, a, L.g, L.ph)
  if (L.out_kind == OUT_RK) {
    if (L.wpe == 2) {
      if (L.fast) WL2_FUSED(OUT_RK, 2, 0, 0); else WL2_FUSED(OUT_RK, 2, -1, -1);
    } else {
      if (L.fast) WL2_FUSED(OUT_RK, 1, 0, 0); else WL2_FUSED(OUT_RK, 1, -1, -1);
    }
  } else {
    if (L.wpe == 2) {
      if (L.fast) WL2_FUSED(OUT_WRITE, 2, 0, 0); else WL2_FUSED(OUT_WRITE, 2, -1, -1);
    } else {
      if (L.fast) WL2_FUSED(OUT_WRITE, 1, 0, 0); else WL2_FUSED(OUT_WRITE, 1, -1, -1);
    }
  }
#undef WL2_FUSED
  return hipGetLastError();
}

hipError_t fused3d_fix(const FusedLaunch& L) {
  const FusedArgs a = make_args(L);
  const dim3 fg(1024), fb(128);
#define WL2_FIX(O, S, H) \
  hipLaunchKernelGGL((weno_fix3d_kernel<O, S, H>), fg, fb, 0, L.stream, a, L.g, L.ph)
  if (L.out_kind == OUT_RK) {
    if (L.fast) WL2_FIX(OUT_RK, 0, 0); else WL2_FIX(OUT_RK, -1, -1);
  } else {
    if (L.fast) WL2_FIX(OUT_WRITE, 0, 0); else WL2_FIX(OUT_WRITE, -1, -1);
  }
#undef WL2_FIX
  return hipGetLastError();
}

}  // namespace wl2
