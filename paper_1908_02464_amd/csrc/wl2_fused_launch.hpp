// Launch interface of the fused 3D stage kernels, which live in a
// translation unit of their own (wl2_fused3d.hip): the heaviest compile of the
// library, built in parallel with the others.
#pragma once
#include <hip/hip_runtime.h>

#include "wl2_device.hpp"

namespace wl2 {

// Column tile of the fused kernel: FT_X x FT_Y cells per workgroup in x, y.
constexpr int FT_X = 16, FT_Y = 15;

struct FusedLaunch {
  const double* Uk;
  double* out;
  const double* Un;
  StepCtl* ctl;
  StepCtl* cfl;  // RK stage: fold the CFL speed of the new state into it (or null)
  unsigned long long* list;
  unsigned int* list_n;      // this stage's list counter
  unsigned int* list_clear;  // the next stage's, zeroed by the correction kernel
  unsigned int* counts;      // entries each stage-kernel workgroup listed in its
                             // region of `list` (fused3d_count_entries of them)
  unsigned int* offs;        // their exclusive prefix sums (one more entry)
  double rk_a, rk_b;
  int out_kind;  // OUT_WRITE or OUT_RK
  int zc;        // z planes per workgroup
  int wpe;       // 1 or 2 waves per SIMD
  double* fo3;   // face changes of the x, y, z faces, 5 values each (face-once
                 // corrections: every face WENO, or the face lists), or null:
                 // the per-cell kernel
  unsigned int* flist;        // face lists (fused3d_flist_entries of them), or null
  unsigned int* counts_f;     // faces each workgroup listed, per direction
  unsigned int* offs_f;       // their exclusive prefix sums (one more entry)
  int n[3];
  KGrid g;
  KPhys ph;
  hipStream_t stream;
};

// The launches of one fused stage, in stream order: the fused stage kernel
// and the nonlinear corrections.  The list counter of a stage is cleared by
// the previous stage's correction kernel; fused3d_reset clears both counters
// (before the first stage, or after a failed launch).
hipError_t fused3d_reset(const FusedLaunch& L);
hipError_t fused3d_main(const FusedLaunch& L);
hipError_t fused3d_fix(const FusedLaunch& L);
// Doubles of the face buffer (FusedLaunch::fo3) of an n[0] x n[1] x n[2] grid.
size_t fused3d_face_doubles(const int n[3]);
// Entries of the per-workgroup count array (FusedLaunch::counts): enough for
// any z chunk (one workgroup per column tile and plane at most).
inline size_t fused3d_count_entries(const int n[3]) {
  return (size_t)((n[0] + FT_X - 1) / FT_X) * ((n[1] + FT_Y - 1) / FT_Y) * n[2];
}
// Entries of the face lists (FusedLaunch::flist): the faces of the three
// directions, each direction's faces once.
inline size_t fused3d_flist_entries(const int n[3]) {
  const size_t nx = n[0], ny = n[1], nz = n[2];
  return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1);
}

}  // namespace wl2
