// Host-side construction of the kernel descriptors of one grid, shared by the
// single-grid context and the batch engine so both derive identical constants.
#pragma once
#include <cmath>
#include "../../include/weno_l2is.h"
#include "wl2_device.hpp"

namespace wl2 {

inline int grid_dim(int ny, int nz) { return nz > 1 ? 3 : (ny > 1 ? 2 : 1); }

inline void fill_grid_desc(const int n[3], int dim, double dx, double gamma,
                           const weno_l2is_params& p, KGrid& g, KPhys& ph) {
  for (int d = 0; d < 3; ++d) {
    g.n[d] = n[d];
    g.bc_lo[d] = p.bc[2 * d];
    g.bc_hi[d] = p.bc[2 * d + 1];
  }
  g.stride[0] = 1;
  g.stride[1] = n[0];
  g.stride[2] = (long long)n[0] * n[1];
  g.ncell = (long long)n[0] * n[1] * n[2];
  g.inflow = nullptr;  // set by the owner of the inflow state
  g.ygh[0] = g.ygh[1] = nullptr;  // set by the owner of the y ghost rows
  ph.gamma = gamma;
  ph.gm1 = gamma - 1.0;
  ph.dx = dx;
  ph.inv_dx = 1.0 / dx;
  ph.cfl = p.cfl;
  ph.c_reg = p.c_reg;
  ph.eps_w = p.eps_weno;
  for (int d = 0; d < 3; ++d) {
    double e = p.thr_C;
    const double r = dx / p.thr_L[d];
    for (int k = 0; k < p.thr_alpha; ++k) e *= r;  // C (dx/L)^alpha, Eq.(35)
    ph.eps_thr[d] = (d < dim) ? e : 0.0;
  }
  ph.split = p.split;
  ph.hybrid = p.hybrid;
  ph.weights = p.weights;
}

// Argument checks shared by every entry point that takes a grid.
inline int validate_grid(int nx, int ny, int nz, double dx, double gamma,
                         const weno_l2is_params* p) {
  if (!p) return WL2_E_NULL;
  if (nx < 1 || ny < 1 || nz < 1) return WL2_E_SHAPE;
  if (nz > 1 && ny < 2) return WL2_E_SHAPE;
  // correction lists count and address cells with 32 bits
  if ((long long)nx * ny * nz > 0xffffffffLL) return WL2_E_SHAPE;
  if (!(dx > 0.0) || !(dx < 1e300) || !(gamma > 1.0) || !(gamma < 1e300)) return WL2_E_PARAM;
  if (!(p->cfl > 0.0) || !(p->c_reg >= 0.0) || !(p->eps_weno >= 0.0) || !(p->thr_C >= 0.0) ||
      p->thr_alpha < 0 || p->thr_alpha > 64)
    return WL2_E_PARAM;
  if (p->split < 0 || p->split > 2 || p->hybrid < 0 || p->hybrid > 3) return WL2_E_PARAM;
  if (p->weights < WL2_W_L2IS || p->weights > WL2_W_IS_B01) return WL2_E_PARAM;
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(p->bgeom[i])) return WL2_E_PARAM;
  const int dim = grid_dim(ny, nz);
  const int n[3] = {nx, ny, nz};
  for (int d = 0; d < dim; ++d) {
    const int lo = p->bc[2 * d], hi = p->bc[2 * d + 1];
    if (lo < 0 || lo > 5 || hi < 0 || hi > 5 || hi == WL2_BC_INFLOW) return WL2_E_BC;
    // state sides: the y sides of a 2D grid only
    const bool st = lo >= WL2_BC_STATE_WALL || hi >= WL2_BC_STATE_WALL;
    if (st && (d != 1 || dim != 2)) return WL2_E_BC;
    // inflow: the x- side of a 1D or 2D grid only
    if (lo == WL2_BC_INFLOW && (d != 0 || dim == 3)) return WL2_E_BC;
    if ((lo == WL2_BC_PERIODIC) != (hi == WL2_BC_PERIODIC)) return WL2_E_BC;
    if ((lo == WL2_BC_REFLECTIVE || hi == WL2_BC_REFLECTIVE) && n[d] < 3) return WL2_E_BC;
    if (!(p->thr_L[d] > 0.0)) return WL2_E_PARAM;
  }
  return WL2_OK;
}

}  // namespace wl2
