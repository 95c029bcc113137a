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
  a.counts = L.counts;
  a.offs = L.offs;
  a.cfl = L.out_kind == OUT_RK ? L.cfl : nullptr;
  a.flist = L.flist;
  a.counts_f = L.counts_f;
  a.offs_f = L.offs_f;
  a.D = L.fo3;
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

// Compile-time scheme builds (the splitting and switch folded in, no
// register spills) for the paper's default (LLF, per-field switch) and for
// the schemes the benchmark and the robustness runs use: every face WENO,
// every face linear, Roe-speed splitting.  Any other combination, and the
// one-wave-per-SIMD budget of those, takes the build that reads the scheme
// at run time.  The arithmetic is the same source either way.
hipError_t fused3d_main(const FusedLaunch& L) {
  const FusedArgs a = make_args(L);
  const long long nzc = (L.n[2] + a.zc - 1) / a.zc;
  const long long blocks = (long long)a.tiles_x * a.tiles_y * nzc;
  if (a.zc < 1 || blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 gr((unsigned)blocks), bl(FT_THREADS);
  const int sp = L.ph.split, hy = L.ph.hybrid;
  const bool dflt = sp == SPLIT_LLF && hy == HYB_PER_FIELD;
#define WL2_FUSED(O, W, S, H) \
  hipLaunchKernelGGL((fused3d_kernel<O, W, S, H>), gr, bl, 0, L.stream, a, L.g, L.ph)
#define WL2_FUSED_SCHEMES(O)                                                         \
  do {                                                                               \
    if (L.wpe != 2) {                                                                \
      if (dflt) WL2_FUSED(O, 1, SPLIT_LLF, HYB_PER_FIELD);                           \
      else WL2_FUSED(O, 1, -1, -1);                                                  \
    } else if (dflt) {                                                               \
      WL2_FUSED(O, 2, SPLIT_LLF, HYB_PER_FIELD);                                     \
    } else if (sp == SPLIT_LLF && hy == HYB_WENO_ONLY) {                             \
      WL2_FUSED(O, 2, SPLIT_LLF, HYB_WENO_ONLY);                                     \
    } else if (sp == SPLIT_LLF && hy == HYB_LINEAR_ONLY) {                           \
      WL2_FUSED(O, 2, SPLIT_LLF, HYB_LINEAR_ONLY);                                   \
    } else if (sp == SPLIT_ROE && hy == HYB_PER_FIELD) {                             \
      WL2_FUSED(O, 2, SPLIT_ROE, HYB_PER_FIELD);                                     \
    } else {                                                                         \
      WL2_FUSED(O, 2, -1, -1);                                                       \
    }                                                                                \
  } while (0)
  if (L.out_kind == OUT_RK) WL2_FUSED_SCHEMES(OUT_RK);
  else WL2_FUSED_SCHEMES(OUT_WRITE);
#undef WL2_FUSED_SCHEMES
#undef WL2_FUSED
  return hipGetLastError();
}

size_t fused3d_face_doubles(const int n[3]) {
  const size_t nx = n[0], ny = n[1], nz = n[2];
  return 5 * ((nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1));
}

// Every face WENO with a face buffer: each face's change once (three
// launches, one per direction), then the per-cell sums.
template <int O, int W>
static hipError_t fix_face_once(const FusedLaunch& L, const FusedArgs& a) {
  const long long nx = L.n[0], ny = L.n[1], nz = L.n[2];
  const long long nfx = (nx + 1) * ny * nz, nfy = nx * (ny + 1) * nz, nfz = nx * ny * (nz + 1);
  double* Dx = L.fo3;
  double* Dy = Dx + 5 * nfx;
  double* Dz = Dy + 5 * nfy;
  const auto blocks = [](long long n, int t) {
    const long long b = (n + t - 1) / t;
    return dim3((unsigned)(b < (1ll << 20) ? b : (1ll << 20)));
  };
  hipLaunchKernelGGL((weno_face3d_kernel<O, 0, SPLIT_LLF, HYB_WENO_ONLY, W>), blocks(nfx, 128), dim3(128), 0,
                     L.stream, a, L.g, L.ph, Dx);
  hipLaunchKernelGGL((weno_face3d_kernel<O, 1, SPLIT_LLF, HYB_WENO_ONLY, W>), blocks(nfy, 128), dim3(128), 0,
                     L.stream, a, L.g, L.ph, Dy);
  hipLaunchKernelGGL((weno_face3d_kernel<O, 2, SPLIT_LLF, HYB_WENO_ONLY, W>), blocks(nfz, 128), dim3(128), 0,
                     L.stream, a, L.g, L.ph, Dz);
  hipLaunchKernelGGL((weno_sum3d_kernel<O>), blocks(nx * ny * nz, 256), dim3(256), 0, L.stream, a, L.g,
                     L.ph, Dx, Dy, Dz);
  return hipGetLastError();
}

// Face lists: the offsets of both lists (one small launch), each listed
// face's change once into the face buffer (one launch for the three lists),
// then the listed cells' sums.
template <int O>
static hipError_t fix_face_lists(const FusedLaunch& L, const FusedArgs& a) {
  const int sp = L.ph.split, hy = L.ph.hybrid;
  const bool w0 = L.ph.weights == W_L2IS;
  const int nreg = a.tiles_x * a.tiles_y * ((L.n[2] + a.zc - 1) / a.zc);
  hipLaunchKernelGGL(list_scan2_kernel, dim3(1), dim3(1024), 0, L.stream, a, nreg);
#define WL2_FL(S, H, W) \
  hipLaunchKernelGGL((weno_flist3d_kernel<O, S, H, W>), dim3(1024), dim3(128), 0, L.stream, a, L.g, L.ph)
  if (w0 && sp == SPLIT_LLF && hy == HYB_PER_FIELD) WL2_FL(SPLIT_LLF, HYB_PER_FIELD, W_L2IS);
  else if (w0 && sp == SPLIT_ROE && hy == HYB_PER_FIELD) WL2_FL(SPLIT_ROE, HYB_PER_FIELD, W_L2IS);
  else WL2_FL(-1, -1, -1);
#undef WL2_FL
  hipLaunchKernelGGL((weno_sumlist3d_kernel<O>), dim3(1024), dim3(256), 0, L.stream, a, L.g, L.ph);
  return hipGetLastError();
}

// The correction kernels have builds for the weighting of Eq.(28) fixed at
// compile time; the comparison weightings take builds that read it at run
// time.  (A run-time choice keeps the values of all three in registers: the
// every-face-WENO face kernel then needs more than 256 VGPRs and runs one
// wave per SIMD, 1.6 against 1.2 ms per launch at 256^3.)
hipError_t fused3d_fix(const FusedLaunch& L) {
  const FusedArgs a = make_args(L);
  const dim3 fg(1024), fb(128);
  const int sp = L.ph.split, hy = L.ph.hybrid;
  const bool w0 = L.ph.weights == W_L2IS;
  if (L.fo3 != nullptr && sp == SPLIT_LLF && hy == HYB_WENO_ONLY) {
    if (L.out_kind == OUT_RK) return w0 ? fix_face_once<OUT_RK, W_L2IS>(L, a) : fix_face_once<OUT_RK, -1>(L, a);
    return w0 ? fix_face_once<OUT_WRITE, W_L2IS>(L, a) : fix_face_once<OUT_WRITE, -1>(L, a);
  }
  if (L.fo3 != nullptr && L.flist != nullptr && hy != HYB_WENO_ONLY)
    return L.out_kind == OUT_RK ? fix_face_lists<OUT_RK>(L, a) : fix_face_lists<OUT_WRITE>(L, a);
  if (!(sp == SPLIT_LLF && hy == HYB_WENO_ONLY)) {
    // offsets of the per-workgroup list regions (the dense form needs none;
    // up to SCAN_LDS regions the correction kernel forms them itself)
    const int nreg = a.tiles_x * a.tiles_y * ((L.n[2] + a.zc - 1) / a.zc);
    if (nreg > SCAN_LDS)
      hipLaunchKernelGGL(list_scan_kernel, dim3(1), dim3(1024), 0, L.stream, a.counts, nreg, a.offs);
  }
#define WL2_FIX(O, S, H, W) \
  hipLaunchKernelGGL((weno_fix3d_kernel<O, S, H, W>), fg, fb, 0, L.stream, a, L.g, L.ph)
  // every face WENO with LLF splitting has its own build for any weighting:
  // the stage kernel's build for it lists no cell, and the correction
  // kernel's build for it walks every cell
#define WL2_FIX_SCHEMES(O)                                                                  \
  do {                                                                                      \
    if (w0 && sp == SPLIT_LLF && hy == HYB_PER_FIELD) WL2_FIX(O, SPLIT_LLF, HYB_PER_FIELD, W_L2IS); \
    else if (w0 && sp == SPLIT_LLF && hy == HYB_WENO_ONLY) WL2_FIX(O, SPLIT_LLF, HYB_WENO_ONLY, W_L2IS); \
    else if (sp == SPLIT_LLF && hy == HYB_WENO_ONLY) WL2_FIX(O, SPLIT_LLF, HYB_WENO_ONLY, -1);  \
    else if (w0 && sp == SPLIT_ROE && hy == HYB_PER_FIELD) WL2_FIX(O, SPLIT_ROE, HYB_PER_FIELD, W_L2IS); \
    else WL2_FIX(O, -1, -1, -1);                                                            \
  } while (0)
  if (L.out_kind == OUT_RK) WL2_FIX_SCHEMES(OUT_RK);
  else WL2_FIX_SCHEMES(OUT_WRITE);
#undef WL2_FIX_SCHEMES
#undef WL2_FIX
  return hipGetLastError();
}

}  // namespace wl2
