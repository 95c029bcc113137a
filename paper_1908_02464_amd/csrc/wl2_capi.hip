// Host side of the C ABI declared in include/weno_l2is.h: argument
// validation, context and scratch management, kernel dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/weno_l2is.h"
#include "wl2_aux.hpp"
#include "wl2_desc.hpp"
#include "wl2_fused_launch.hpp"
#include "wl2_row_launch.hpp"
#include "wl2_kernels.hpp"

using namespace wl2;

struct weno_l2is_ctx {
  int n[3];
  int dim, nvar;
  long long ncell;
  double dx, gamma;
  weno_l2is_params p;
  hipStream_t stream;
  int device;
  double* U1;
  double* U2;
  double* acc;
  unsigned long long* list;  // cells next to faces needing the WENO flux (fused kernels)
  double* fo_D = nullptr;          // 2D face-once corrections: face changes per list entry
  unsigned int* fo_map = nullptr;  // and the cell -> list entry map (null: per-cell kernel)
  double* fo3 = nullptr;           // 3D: each face's change (face-once corrections)
  unsigned int* flist = nullptr;   // 3D hybrid: faces needing the WENO flux
  unsigned int* counts = nullptr;  // 3D: entries each stage-kernel workgroup listed
  double* inflow = nullptr;        // x- inflow side: ghost state [nvar][ny*nz]
  double* ygh = nullptr;           // y state sides: ghost rows of both, [side][layer][nvar][nx]
  bool inflow_set = false;         // weno_l2is_set_inflow has been called
  double inflow_speed = 0.0;       // CFL speed sum_d(|u_d| + c), max over the inflow states
  StepCtl* ctl;
  KGrid g;
  KPhys ph;
  int path;    // WL2_PATH_*
  int zchunk;  // fused kernel: planes per workgroup (0 = automatic)
  int wpe;     // fused kernel: target waves per SIMD (1 or 2)
  int n_cu = 0;  // compute units of the device (0: unknown)
  // correction-list counters (ctl->list_n[2]): the stage in flight uses
  // list_par, its correction kernel clears the other one for the next stage;
  // both are cleared before the first stage and after a failed launch
  int list_par = 0;
  bool list_dirty = true;
  // optional per-launch event timing
  bool timing;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_used;  // (kernel id, pool index of start event)
  std::vector<std::string> knames;
};

namespace {

constexpr int SEG = 8;  // cells per thread along the sweep

// Timing: bracket a launch with two events of the pool.
struct TimedLaunch {
  weno_l2is_ctx* c;
  int slot;
  TimedLaunch(const weno_l2is_ctx* cc, const char* name) : c(const_cast<weno_l2is_ctx*>(cc)), slot(-1) {
    if (!c->timing) return;
    int id = -1;
    for (size_t i = 0; i < c->knames.size(); ++i)
      if (c->knames[i] == name) id = (int)i;
    if (id < 0) {
      id = (int)c->knames.size();
      c->knames.push_back(name);
    }
    const size_t need = 2 * (c->ev_used.size() + 1);
    while (c->ev_pool.size() < need) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      c->ev_pool.push_back(e);
    }
    slot = (int)(2 * c->ev_used.size());
    c->ev_used.emplace_back(id, slot);
    (void)hipEventRecord(c->ev_pool[slot], c->stream);
  }
  ~TimedLaunch() {
    if (slot >= 0) (void)hipEventRecord(c->ev_pool[slot + 1], c->stream);
  }
};

template <int NV, int DIR, int OUT>
const char* sweep_name() {
  static const char* tab[3][3] = {{"sweep_x_write", "sweep_x_accum", "sweep_x_rk"},
                                  {"sweep_y_write", "sweep_y_accum", "sweep_y_rk"},
                                  {"sweep_z_write", "sweep_z_accum", "sweep_z_rk"}};
  return tab[DIR][OUT];
}

// Do the byte ranges [a, a + na) and [b, b + nb) share a byte?
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

bool overlaps(const double* a, const double* b, size_t n) {
  return overlaps(a, n * sizeof(double), b, n * sizeof(double));
}

int validate(int nx, int ny, int nz, double dx, double gamma, const weno_l2is_params* p) {
  return validate_grid(nx, ny, nz, dx, gamma, p);
}

void fill_desc(weno_l2is_ctx* c) {
  fill_grid_desc(c->n, c->dim, c->dx, c->gamma, c->p, c->g, c->ph);
  c->g.inflow = c->inflow;
  if (c->ygh) {
    const size_t side = (size_t)3 * 4 * c->n[0];
    c->g.ygh[0] = c->p.bc[2] >= WL2_BC_STATE_WALL ? c->ygh : nullptr;
    c->g.ygh[1] = c->p.bc[3] >= WL2_BC_STATE_WALL ? c->ygh + side : nullptr;
  }
}

bool has_state_sides(const weno_l2is_params* p, int dim) {
  return dim == 2 && (p->bc[2] >= WL2_BC_STATE_WALL || p->bc[3] >= WL2_BC_STATE_WALL);
}

// Ghost rows of the y state sides for the state Uk, at the stage time
// t0 + tc dt (tc < 0: the clock's t).
YGhostRule ghost_rule(const weno_l2is_ctx* c) {
  YGhostRule r;
  for (int s = 0; s < 2; ++s)
    for (int v = 0; v < 4; ++v) r.state[s][v] = c->p.bstate[s][v];
  for (int i = 0; i < 4; ++i) r.geom[i] = c->p.bgeom[i];
  return r;
}

hipError_t fill_yghosts(const weno_l2is_ctx* c, const double* Uk, double tc) {
  if (!c->ygh) return hipSuccess;
  const long long n = 2ll * 3 * c->n[0];
  hipLaunchKernelGGL(ghost_fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, Uk,
                     c->g, c->ctl, tc, c->dx, ghost_rule(c), const_cast<double*>(c->g.ygh[0]),
                     const_cast<double*>(c->g.ygh[1]));
  return hipGetLastError();
}

// An inflow side whose ghost state has not been given yet.
bool inflow_missing(const weno_l2is_ctx* c) {
  return c->p.bc[0] == WL2_BC_INFLOW && !c->inflow_set;
}

int hip_err(hipError_t e) { return e == hipSuccess ? WL2_OK : WL2_E_HIP; }

template <int NV, int DIR, int OUT>
hipError_t launch_sweep_t(const weno_l2is_ctx* c, const SweepArgs& a) {
  const int n = c->n[DIR];
  const int nseg = (n + SEG - 1) / SEG;
  const long long nthreads = (long long)nseg * (c->ncell / n);
  const long long blocks = (nthreads + SWEEP_BLOCK - 1) / SWEEP_BLOCK;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  TimedLaunch tl(c, sweep_name<NV, DIR, OUT>());
  hipLaunchKernelGGL((sweep_kernel<NV, DIR, SEG, OUT>), dim3((unsigned)blocks), dim3(SWEEP_BLOCK),
                     0, c->stream, a, c->g, c->ph, nseg, nthreads);
  return hipGetLastError();
}

template <int NV, int OUT>
hipError_t launch_sweep_nv(const weno_l2is_ctx* c, int dir, const SweepArgs& a) {
  if (dir == 0) return launch_sweep_t<NV, 0, OUT>(c, a);
  if (NV >= 4 && dir == 1) return launch_sweep_t<NV, (NV >= 4 ? 1 : 0), OUT>(c, a);
  if (NV >= 5 && dir == 2) return launch_sweep_t<NV, (NV >= 5 ? 2 : 0), OUT>(c, a);
  return hipErrorInvalidValue;
}

hipError_t launch_sweep(const weno_l2is_ctx* c, int dir, int out, const SweepArgs& a) {
  switch (c->nvar * 3 + out) {
    case 9 + OUT_WRITE: return launch_sweep_nv<3, OUT_WRITE>(c, dir, a);
    case 9 + OUT_ACCUM: return launch_sweep_nv<3, OUT_ACCUM>(c, dir, a);
    case 9 + OUT_RK: return launch_sweep_nv<3, OUT_RK>(c, dir, a);
    case 12 + OUT_WRITE: return launch_sweep_nv<4, OUT_WRITE>(c, dir, a);
    case 12 + OUT_ACCUM: return launch_sweep_nv<4, OUT_ACCUM>(c, dir, a);
    case 12 + OUT_RK: return launch_sweep_nv<4, OUT_RK>(c, dir, a);
    case 15 + OUT_WRITE: return launch_sweep_nv<5, OUT_WRITE>(c, dir, a);
    case 15 + OUT_ACCUM: return launch_sweep_nv<5, OUT_ACCUM>(c, dir, a);
    case 15 + OUT_RK: return launch_sweep_nv<5, OUT_RK>(c, dir, a);
  }
  return hipErrorInvalidValue;
}

unsigned red_blocks(long long ncell) {
  long long b = (ncell + RED_BLOCK - 1) / RED_BLOCK;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// dt of the next step: the CFL reduction of U (skipped when the previous
// stage kernel already folded the maximum of U into the control word), then
// the finalisation.
hipError_t launch_cfl(const weno_l2is_ctx* c, const double* U, double dt_fixed, int use_clock,
                      bool reduced = false) {
  if (dt_fixed <= 0.0 && !reduced) {
    const unsigned b = red_blocks(c->ncell);
    TimedLaunch tl(c, "cfl_reduce");
    switch (c->nvar) {
      case 3: hipLaunchKernelGGL(cfl_reduce_kernel<3>, dim3(b), dim3(RED_BLOCK), 0, c->stream, U, c->ncell, c->gamma, c->ctl); break;
      case 4: hipLaunchKernelGGL(cfl_reduce_kernel<4>, dim3(b), dim3(RED_BLOCK), 0, c->stream, U, c->ncell, c->gamma, c->ctl); break;
      default: hipLaunchKernelGGL(cfl_reduce_kernel<5>, dim3(b), dim3(RED_BLOCK), 0, c->stream, U, c->ncell, c->gamma, c->ctl); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    TimedLaunch tl(c, "finalize_dt");
    hipLaunchKernelGGL(finalize_dt_kernel, dim3(1), dim3(64), 0, c->stream, c->ctl, c->p.cfl * c->dx,
                       dt_fixed, use_clock, c->inflow_speed);
  }
  return hipGetLastError();
}

// Global LF speeds of U: per-block maxima into the slots, then the maximum
// over the slots into ctl->lf_bits (the slots are zero between reductions:
// the control block starts zeroed and the finalize kernel clears them).
// With y state sides the reduction's launch also fills their ghost rows for
// stage time tc (as fill_yghosts).
hipError_t launch_lf(const weno_l2is_ctx* c, const double* U, double tc) {
  const unsigned b = red_blocks(c->ncell);
  double* lo = const_cast<double*>(c->g.ygh[0]);
  double* hi = const_cast<double*>(c->g.ygh[1]);
  const YGhostRule r = ghost_rule(c);
#define WL2_LFR(NV, GH)                                                                      \
  hipLaunchKernelGGL((lf_reduce_kernel<NV, GH>), dim3(b), dim3(RED_BLOCK), 0, c->stream, U, \
                     c->ncell, c->gamma, c->ctl, c->g, tc, c->dx, r, lo, hi)
  if (c->ygh) {
    if (c->nvar != 4) return hipErrorInvalidValue;
    WL2_LFR(4, true);
  } else if (c->nvar == 3) {
    WL2_LFR(3, false);
  } else if (c->nvar == 4) {
    WL2_LFR(4, false);
  } else {
    WL2_LFR(5, false);
  }
#undef WL2_LFR
  hipLaunchKernelGGL(lf_finalize_kernel, dim3(1), dim3(64), 0, c->stream, c->ctl, c->nvar);
  return hipGetLastError();
}

bool use_fused(const weno_l2is_ctx* c) { return c->dim == 3 && c->path != WL2_PATH_SWEEPS; }
bool use_row(const weno_l2is_ctx* c) { return c->dim <= 2 && c->path != WL2_PATH_SWEEPS; }
// advance() of a small 1D grid runs in one single-workgroup launch (not with
// global Lax-Friedrichs speeds, which need a grid-wide reduction per stage)
bool use_row_steps(const weno_l2is_ctx* c) {
  if (c->p.bc[0] == WL2_BC_INFLOW) return false;  // its time step has no inflow speed
  return c->dim == 1 && use_row(c) && c->n[0] <= ROW_STEPS_MAX_CELLS && c->p.split != WL2_SPLIT_LF;
}

// 2D grids from this many cells correct their flagged faces once each (two
// launches) instead of once per adjacent listed cell (one launch): the
// lists of large grids are long enough for the halved work to outweigh the
// extra launch.
constexpr long long FACE_ONCE_MIN_CELLS = 1ll << 17;

// Rows per work item of the 1D/2D kernel: the tuned value, else the largest
// of 6 .. 2 that still gives >= 1536 items, three quarters of the 2048
// wavefronts the chip holds at once (measured: 6 rows at 1024^2 and 2048^2,
// 3 at 512^2, 2 at 256^2; longer marches amortise the six-cell start of a
// column, more items fill the chip).
int row_ych(const weno_l2is_ctx* c) {
  if (c->dim == 1) return 1;
  const int cap = ROW_MAX_YCH < c->n[1] ? ROW_MAX_YCH : c->n[1];
  if (c->zchunk > 0) return c->zchunk < cap ? c->zchunk : cap;
  // One wavefront per item and two per SIMD: 2048 items run at once.  If
  // the grid fits one such round with at most 12 rows per item, the fewest
  // rows that do (the most parallel single round); otherwise 11 rows (fewer
  // warm-up rows per row computed; items then run in several rounds).
  constexpr long long ROUND = 2048;
  const long long tiles = (c->n[0] + ROW_TILE - 1) / ROW_TILE;
  const int ymax = 12 < cap ? 12 : cap;
  for (int y = 2; y <= ymax; ++y)
    if (tiles * ((c->n[1] + y - 1) / y) <= ROUND) return y;
  return 11 < cap ? 11 : cap;
}

// The counters of the next stage launch, clearing both if needed.
struct ListTurn {
  weno_l2is_ctx* c;
  unsigned int* cur;
  unsigned int* next;
  bool reset;
  explicit ListTurn(const weno_l2is_ctx* cc) : c(const_cast<weno_l2is_ctx*>(cc)) {
    cur = &c->ctl->list_n[c->list_par];
    next = &c->ctl->list_n[c->list_par ^ 1];
    reset = c->list_dirty;
  }
  // after the stage's launches: flip on success, clear both next time if not
  hipError_t done(hipError_t e) {
    if (e == hipSuccess) {
      c->list_par ^= 1;
      c->list_dirty = false;
    } else {
      c->list_dirty = true;
    }
    return e;
  }
};

hipError_t launch_row(const weno_l2is_ctx* c, int out_kind, const double* Uk, double* out,
                      const double* Un, double ra, double rb, bool fold_cfl = false,
                      bool kclock = false) {
  ListTurn turn(c);
  RowLaunch L;
  L.Uk = Uk;
  L.out = out;
  L.Un = Un;
  L.ctl = c->ctl;
  L.rk_a = ra;
  L.rk_b = rb;
  L.out_kind = out_kind;
  L.ych = row_ych(c);
  L.fast = c->p.hybrid != WL2_HYB_PER_FIELD ? 0
           : c->p.split == WL2_SPLIT_LLF   ? 1
           : c->p.split == WL2_SPLIT_LF    ? 2
                                           : 0;
  L.nvar = c->nvar;
  L.list = c->list;
  L.list_n = turn.cur;
  L.list_clear = turn.next;
  L.cfl = fold_cfl ? c->ctl : nullptr;
  L.clock = kclock ? c->ctl : nullptr;
  L.cfl_dx = c->p.cfl * c->dx;
  L.s_floor = c->inflow_speed;
  L.fo_D = c->path == WL2_PATH_FUSED_CELLS ? nullptr : c->fo_D;
  L.fo_map = c->fo_map;
  L.fo_cap = (unsigned int)c->ncell;
  L.g = c->g;
  L.ph = c->ph;
  L.stream = c->stream;
  hipError_t e = turn.reset ? row_reset(L) : hipSuccess;
  if (e != hipSuccess) return turn.done(e);
  {
    TimedLaunch tl(c, out_kind == OUT_RK ? "row_rk" : "row_rhs");
    if ((e = row_launch(L)) != hipSuccess) return turn.done(e);
  }
  TimedLaunch tl(c, "row_fix");
  return turn.done(row_fix(L));
}

// Planes per workgroup of the fused 3D stage kernel (the tuned value, or a
// choice from the grid's shape).  The workgroups run in rounds of as many as
// the chip holds at once (two per CU, one with the one-wave budget); a last
// round that is partly empty idles CUs for a whole march, and every march
// pays a warm-up of about three planes.  So among balanced chunks of 16 to
// 128 planes (zc = ceil(nz / k)) giving at least three rounds, the choice
// maximizes (fill of the rounds) x zc / (zc + 3).  Measured against the
// earlier rule (the longest power-of-two fraction of nz giving 2048
// workgroups), Mcell-updates/s per stage: 512^3 19.2 -> 20.5 (103 planes
// instead of 256), 640^3 19.8 -> 20.6 (80 instead of 320), 256^3 +1 % (37
// instead of 32), 384^3 unchanged (96).  Grids too small for three rounds
// of 16-plane chunks halve the chunk from nz while that adds workgroups.
int fused_zchunk(const weno_l2is_ctx* c) {
  const int nz = c->n[2];
  if (c->zchunk > 0) return c->zchunk < nz ? c->zchunk : nz;
  const long long tiles = (long long)((c->n[0] + FT_X - 1) / FT_X) * ((c->n[1] + FT_Y - 1) / FT_Y);
  const long long cap = (long long)(c->n_cu > 0 ? c->n_cu : 256) * (c->wpe == 1 ? 1 : 2);
  const auto halving = [&]() {
    int zc = nz;
    while (zc > 16 && tiles * ((nz + zc - 1) / zc) < 2048) zc = (zc + 1) / 2;
    return zc;
  };
  if (tiles * ((nz + 15) / 16) < 3 * cap) return halving();
  int best = 0;
  double best_score = -1.0;
  for (int k = (nz + 127) / 128; k <= nz / 16; ++k) {
    const int zc = (nz + k - 1) / k;
    const long long wg = tiles * ((nz + zc - 1) / zc);
    if (zc < 16 || zc > 128 || wg < 3 * cap) continue;
    const long long rounds = (wg + cap - 1) / cap;
    const double score = (double)wg / (double)(rounds * cap) * zc / (zc + 3.0);
    if (score > best_score + 1e-12) {
      best_score = score;
      best = zc;
    }
  }
  return best > 0 ? best : halving();  // (no balanced chunk of 16..128 planes)
}

hipError_t launch_fused(const weno_l2is_ctx* c, int out_kind, const double* Uk, double* out,
                        const double* Un, double ra, double rb, bool fold_cfl = false) {
  ListTurn turn(c);
  FusedLaunch L;
  L.Uk = Uk;
  L.out = out;
  L.Un = Un;
  L.ctl = c->ctl;
  L.cfl = fold_cfl ? c->ctl : nullptr;
  L.list = c->list;
  L.list_n = turn.cur;
  L.list_clear = turn.next;
  L.rk_a = ra;
  L.rk_b = rb;
  L.out_kind = out_kind;
  L.zc = fused_zchunk(c);
  L.wpe = c->wpe;  // the scheme's build is chosen from L.ph
  L.fo3 = c->path == WL2_PATH_FUSED_CELLS ? nullptr : c->fo3;
  L.flist = c->path == WL2_PATH_FUSED_CELLS ? nullptr : c->flist;
  const size_t ce = fused3d_count_entries(c->n);
  L.counts = c->counts;
  L.offs = c->counts ? c->counts + ce : nullptr;
  L.counts_f = c->counts ? c->counts + 2 * ce + 1 : nullptr;
  L.offs_f = c->counts ? c->counts + 5 * ce + 1 : nullptr;
  for (int d = 0; d < 3; ++d) L.n[d] = c->n[d];
  L.g = c->g;
  L.ph = c->ph;
  L.stream = c->stream;
  hipError_t e = turn.reset ? fused3d_reset(L) : hipSuccess;
  if (e != hipSuccess) return turn.done(e);
  {
    TimedLaunch tl(c, out_kind == OUT_RK ? "fused3d_rk" : "fused3d_rhs");
    if ((e = fused3d_main(L)) != hipSuccess) return turn.done(e);
  }
  // nonlinear corrections of the listed cells (an empty list exits at once)
  TimedLaunch tl(c, "weno_fix3d");
  return turn.done(fused3d_fix(L));
}

// dU/dt of the state Uk into out (WRITE then ACCUM over directions).
hipError_t rhs_into(const weno_l2is_ctx* c, const double* Uk, double* out) {
  hipError_t e;
  e = c->p.split == WL2_SPLIT_LF ? launch_lf(c, Uk, -1.0) : fill_yghosts(c, Uk, -1.0);
  if (e != hipSuccess) return e;
  if (use_fused(c)) return launch_fused(c, OUT_WRITE, Uk, out, nullptr, 0.0, 1.0);
  if (use_row(c)) return launch_row(c, OUT_WRITE, Uk, out, nullptr, 0.0, 1.0);
  for (int d = 0; d < c->dim; ++d) {
    SweepArgs a{Uk, out, nullptr, nullptr, c->ctl, 0.0, 1.0};
    if ((e = launch_sweep(c, d, d == 0 ? OUT_WRITE : OUT_ACCUM, a)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// One RK stage: out = a Un + b (Uk + dt L(Uk)).  fold_cfl (fused 3D and row
// 1D/2D paths): the stage kernels also fold the CFL maximum of `out` into
// the control word.
// kclock (1D/2D stage 1): the step's dt has not been formed yet; the stage
// kernel forms it (finalize_dt_kernel's rule) and the clock still reads the
// step's start, which the ghost rows take as their time (tc = 0).
hipError_t stage(const weno_l2is_ctx* c, const double* Uk, const double* Un, double* out,
                 double ra, double rb, double tc, bool fold_cfl = false, bool kclock = false) {
  hipError_t e;
  const double tg = kclock ? -1.0 : tc;  // -1: the clock's t
  e = c->p.split == WL2_SPLIT_LF ? launch_lf(c, Uk, tg) : fill_yghosts(c, Uk, tg);
  if (e != hipSuccess) return e;
  if (use_fused(c)) return launch_fused(c, OUT_RK, Uk, out, Un, ra, rb, fold_cfl);
  if (use_row(c)) return launch_row(c, OUT_RK, Uk, out, Un, ra, rb, fold_cfl, kclock);
  for (int d = 0; d < c->dim - 1; ++d) {
    SweepArgs a{Uk, c->acc, nullptr, nullptr, c->ctl, 0.0, 1.0};
    if ((e = launch_sweep(c, d, d == 0 ? OUT_WRITE : OUT_ACCUM, a)) != hipSuccess) return e;
  }
  SweepArgs a{Uk, out, c->dim > 1 ? c->acc : nullptr, Un, c->ctl, ra, rb};
  return launch_sweep(c, c->dim - 1, OUT_RK, a);
}

hipError_t rk3(const weno_l2is_ctx* c, double* U, bool fold_cfl = false, bool kclock = false) {
  hipError_t e;
  // the stages at the times t0, t0 + dt, t0 + dt/2 of the Shu-Osher form
  if ((e = stage(c, U, nullptr, c->U1, 0.0, 1.0, 0.0, false, kclock)) != hipSuccess) return e;
  if ((e = stage(c, c->U1, U, c->U2, 0.75, 0.25, 1.0)) != hipSuccess) return e;
  return stage(c, c->U2, U, U, 1.0 / 3.0, 2.0 / 3.0, 0.5, fold_cfl);
}

std::mutex g_cache_mu;
// key: grid shape, device, whether the context holds y state-side ghost rows
std::map<std::tuple<int, int, int, int, int>, weno_l2is_ctx*> g_cache;

}  // namespace

// ------------------------------------------------ allocation-free rhs
// Static scratch of weno_l2is_rhs_noalloc: one array per GPU, in the code
// object.  Host code never uses the name as an address: the device address
// of each GPU's copy comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char wl2_noalloc_scratch[WL2_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's scratch (null on failure).
void* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(wl2_noalloc_scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_noalloc_ptr[dev] = p;
  }
  return g_noalloc_ptr[dev];
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Scratch of one right-hand side with per-cell corrections: control block,
// (3D) the per-workgroup list counts and their offsets, the correction list.
size_t noalloc_bytes(const int n[3], int dim) {
  const size_t ncell = (size_t)n[0] * n[1] * n[2];
  size_t b = align256(sizeof(StepCtl));
  if (dim == 3) b += align256(sizeof(unsigned int) * (2 * fused3d_count_entries(n) + 1));
  return b + sizeof(unsigned long long) * ncell;
}

__global__ void zero_words_kernel(unsigned long long* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

}  // namespace

extern "C" {

int weno_l2is_params_default(weno_l2is_params* p, int nx, int ny, int nz, double dx) {
  if (!p) return WL2_E_NULL;
  if (nx < 1 || ny < 1 || nz < 1) return WL2_E_SHAPE;
  if (!(dx > 0.0)) return WL2_E_PARAM;
  std::memset(p, 0, sizeof(*p));
  p->cfl = 0.5;
  p->c_reg = 1.0;
  p->eps_weno = 1e-20;
  p->thr_C = 1.0;
  p->thr_alpha = 3;
  p->split = WL2_SPLIT_LLF;
  p->hybrid = WL2_HYB_PER_FIELD;
  for (int i = 0; i < 6; ++i) p->bc[i] = WL2_BC_TRANSMISSIVE;
  p->thr_L[0] = nx * dx;
  p->thr_L[1] = ny * dx;
  p->thr_L[2] = nz * dx;
  p->weights = WL2_W_L2IS;
  return WL2_OK;
}

int weno_l2is_create(int nx, int ny, int nz, double dx, double gamma, const weno_l2is_params* p,
                     void* hip_stream, weno_l2is_ctx** out) {
  if (!out) return WL2_E_NULL;
  *out = nullptr;
  int rc = validate(nx, ny, nz, dx, gamma, p);
  if (rc) return rc;
  weno_l2is_ctx* c = new (std::nothrow) weno_l2is_ctx();
  if (!c) return WL2_E_NOMEM;
  c->n[0] = nx;
  c->n[1] = ny;
  c->n[2] = nz;
  c->dim = nz > 1 ? 3 : (ny > 1 ? 2 : 1);
  c->nvar = c->dim + 2;
  c->ncell = (long long)nx * ny * nz;
  c->dx = dx;
  c->gamma = gamma;
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  c->wpe = 2;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return WL2_E_HIP;
  }
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
    (void)hipGetLastError();
    c->n_cu = 0;
  }
  fill_desc(c);
  const size_t bytes = sizeof(double) * (size_t)c->ncell * c->nvar;
  bool ok = hipMalloc(&c->U1, bytes) == hipSuccess && hipMalloc(&c->U2, bytes) == hipSuccess &&
            hipMalloc(&c->acc, bytes) == hipSuccess &&
            hipMalloc(&c->ctl, sizeof(StepCtl)) == hipSuccess;
  if (ok) ok = hipMalloc(&c->list, sizeof(unsigned long long) * (size_t)c->ncell) == hipSuccess;
  if (ok && c->dim == 2 && c->ncell >= FACE_ONCE_MIN_CELLS && c->ncell <= 0xffffffffll)
    ok = hipMalloc(&c->fo_D, sizeof(double) * 2 * c->nvar * (size_t)c->ncell) == hipSuccess &&
         hipMalloc(&c->fo_map, sizeof(unsigned int) * (size_t)c->ncell) == hipSuccess &&
         // every map value stays a valid entry index (< ncell) from the start
         hipMemsetAsync(c->fo_map, 0, sizeof(unsigned int) * (size_t)c->ncell, c->stream) == hipSuccess;
  // 3D: the corrections compute each face once into a face buffer (15
  // doubles per cell): every face with every face WENO (LLF splitting), the
  // faces of the face lists (3 entries per cell) with the hybrid switch
  const bool hyb3 = c->dim == 3 && (p->hybrid == WL2_HYB_PER_FIELD || p->hybrid == WL2_HYB_PER_FACE);
  if (ok && c->dim == 3 && ((p->hybrid == WL2_HYB_WENO_ONLY && p->split == WL2_SPLIT_LLF) || hyb3))
    ok = hipMalloc(&c->fo3, sizeof(double) * fused3d_face_doubles(c->n)) == hipSuccess;
  if (ok && hyb3)
    ok = hipMalloc(&c->flist, sizeof(unsigned int) * fused3d_flist_entries(c->n)) == hipSuccess;
  // 3D: per-workgroup counts of the correction list and their prefix sums
  if (ok && p->bc[0] == WL2_BC_INFLOW)
    ok = hipMalloc(&c->inflow, sizeof(double) * c->nvar * (size_t)ny * nz) == hipSuccess;
  if (ok) c->g.inflow = c->inflow;
  // y state sides (2D): three ghost rows per side, refilled every stage
  if (ok && has_state_sides(p, c->dim))
    ok = hipMalloc(&c->ygh, sizeof(double) * 2 * 3 * 4 * (size_t)nx) == hipSuccess;
  if (ok) fill_desc(c);
  // (cell list: counts and offsets; face lists: counts and offsets over
  // three directions)
  if (ok && c->dim == 3)
    ok = hipMalloc(&c->counts, sizeof(unsigned int) * (8 * fused3d_count_entries(c->n) + 2)) ==
         hipSuccess;
  if (ok) ok = hipMemsetAsync(c->ctl, 0, sizeof(StepCtl), c->stream) == hipSuccess;
  if (!ok) {
    (void)hipFree(c->U1);
    (void)hipFree(c->U2);
    (void)hipFree(c->acc);
    (void)hipFree(c->list);
    (void)hipFree(c->fo_D);
    (void)hipFree(c->fo_map);
    (void)hipFree(c->fo3);
    (void)hipFree(c->flist);
    (void)hipFree(c->counts);
    (void)hipFree(c->inflow);
    (void)hipFree(c->ygh);
    (void)hipFree(c->ctl);
    delete c;
    (void)hipGetLastError();
    return WL2_E_NOMEM;
  }
  *out = c;
  return WL2_OK;
}

void weno_l2is_destroy(weno_l2is_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  (void)hipFree(c->U1);
  (void)hipFree(c->U2);
  (void)hipFree(c->acc);
  (void)hipFree(c->list);
  (void)hipFree(c->fo_D);
  (void)hipFree(c->fo_map);
  (void)hipFree(c->fo3);
  (void)hipFree(c->flist);
  (void)hipFree(c->counts);
  (void)hipFree(c->inflow);
  (void)hipFree(c->ygh);
  (void)hipFree(c->ctl);
  delete c;
}

int weno_l2is_set_inflow(weno_l2is_ctx* c, const double* state) {
  if (!c || !state) return WL2_E_NULL;
  if (c->p.bc[0] != WL2_BC_INFLOW || !c->inflow) return WL2_E_BC;
  const size_t rows = (size_t)c->n[1] * c->n[2];
  const size_t bytes = sizeof(double) * c->nvar * rows;
  // the caller's state is checked on the host before it replaces anything:
  // a refused state leaves the ghosts and the inflow speed of the last
  // accepted one in place
  std::vector<double> h((size_t)c->nvar * rows);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpy(h.data(), state, bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return WL2_E_HIP;
  // the time step also bounds the speed of the inflow states (the jet enters
  // at a speed no interior cell has yet): their CFL speed
  double smax = 0.0;
  for (size_t r = 0; r < rows; ++r) {
    const double rho = h[r], E = h[(c->nvar - 1) * rows + r];
    double q = 0.0;
    for (int d = 0; d < c->dim; ++d) {
      const double u = h[(1 + d) * rows + r] / rho;
      q += u * u;
    }
    const double p = (c->gamma - 1.0) * (E - 0.5 * rho * q);
    if (!(rho > 0.0) || !(p > 0.0) || !std::isfinite(E)) return WL2_E_PARAM;
    const double cs = std::sqrt(c->gamma * p / rho);
    double s = 0.0;
    for (int d = 0; d < c->dim; ++d) s += std::fabs(h[(1 + d) * rows + r] / rho) + cs;
    if (s > smax) smax = s;
  }
  e = hipMemcpyAsync(c->inflow, h.data(), bytes, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return WL2_E_HIP;
  c->inflow_speed = smax;
  c->inflow_set = true;
  return WL2_OK;
}

int weno_l2is_rhs_ctx(weno_l2is_ctx* c, const double* U, double* dUdt) {
  if (!c || !U || !dUdt) return WL2_E_NULL;
  if (overlaps(U, dUdt, (size_t)c->nvar * c->ncell)) return WL2_E_PARAM;
  if (inflow_missing(c)) return WL2_E_BC;
  return hip_err(rhs_into(c, U, dUdt));
}

int weno_l2is_rhs(const double* U, int nx, int ny, int nz, double dx, double gamma,
                  const weno_l2is_params* params, double* dUdt) {
  if (!U || !dUdt) return WL2_E_NULL;
  int rc = validate(nx, ny, nz, dx, gamma, params);
  if (rc) return rc;
  if (params->bc[0] == WL2_BC_INFLOW) return WL2_E_BC;  // no context to hold its state
  const size_t nc = (size_t)nx * ny * nz;
  if (overlaps(U, dUdt, (size_t)(2 + (ny > 1) + (nz > 1)) * nc)) return WL2_E_PARAM;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WL2_E_HIP;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto key = std::make_tuple(nx, ny, nz, dev, has_state_sides(params, grid_dim(ny, nz)) ? 1 : 0);
  weno_l2is_ctx* c = nullptr;
  auto it = g_cache.find(key);
  if (it == g_cache.end()) {
    rc = weno_l2is_create(nx, ny, nz, dx, gamma, params, nullptr, &c);
    if (rc) return rc;
    g_cache[key] = c;
  } else {
    c = it->second;
    c->dx = dx;
    c->gamma = gamma;
    c->p = *params;
    fill_desc(c);
  }
  return hip_err(rhs_into(c, U, dUdt));
}

int weno_l2is_rhs_noalloc(const double* U, int nx, int ny, int nz, double dx, double gamma,
                          const weno_l2is_params* params, double* dUdt, void* hip_stream) {
  if (!U || !dUdt) return WL2_E_NULL;
  int rc = validate(nx, ny, nz, dx, gamma, params);
  if (rc) return rc;
  if (params->bc[0] == WL2_BC_INFLOW) return WL2_E_BC;  // no context to hold its state
  const int dim = nz > 1 ? 3 : (ny > 1 ? 2 : 1);
  if (has_state_sides(params, dim)) return WL2_E_BC;  // no scratch for their ghost rows
  const size_t nc = (size_t)nx * ny * nz;
  if (overlaps(U, dUdt, (size_t)(2 + dim) * nc)) return WL2_E_PARAM;
  const int n[3] = {nx, ny, nz};
  if (noalloc_bytes(n, dim) > (size_t)WL2_NOALLOC_SCRATCH_BYTES) return WL2_E_BUDGET;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WL2_E_HIP;
  unsigned char* base = (unsigned char*)noalloc_scratch(dev);
  if (!base) return WL2_E_HIP;
  // a context on the host stack over the scratch: nothing is allocated;
  // the per-cell correction kernels need only the list (no face buffers)
  weno_l2is_ctx c;
  c.n[0] = nx;
  c.n[1] = ny;
  c.n[2] = nz;
  c.dim = dim;
  c.nvar = dim + 2;
  c.ncell = (long long)nc;
  c.dx = dx;
  c.gamma = gamma;
  c.p = *params;
  c.stream = (hipStream_t)hip_stream;
  c.device = dev;
  if (hipDeviceGetAttribute(&c.n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    c.n_cu = 0;
  }
  c.U1 = c.U2 = c.acc = nullptr;
  size_t off = 0;
  c.ctl = (StepCtl*)(base + off);
  off += align256(sizeof(StepCtl));
  if (dim == 3) {
    c.counts = (unsigned int*)(base + off);
    off += align256(sizeof(unsigned int) * (2 * fused3d_count_entries(n) + 1));
  }
  c.list = (unsigned long long*)(base + off);
  c.path = WL2_PATH_FUSED_CELLS;
  c.zchunk = 0;
  c.wpe = 2;
  c.list_par = 0;
  c.list_dirty = true;  // both list counters cleared by the first launch
  c.timing = false;
  fill_desc(&c);
  // the control block starts at zero (a kernel, not a memset: the call may
  // be captured into a graph)
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(256), 0, c.stream,
                     (unsigned long long*)c.ctl, sizeof(StepCtl) / sizeof(unsigned long long));
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = rhs_into(&c, U, dUdt);
  return hip_err(e);
}

int weno_l2is_rhs_release(void) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  int cur = 0, n = 0;
  if (!g_cache.empty() && hipGetDevice(&cur) != hipSuccess) return WL2_E_HIP;
  for (auto& kv : g_cache) {
    // each context's memory belongs to the device it was made on
    if (hipSetDevice(std::get<3>(kv.first)) != hipSuccess) return WL2_E_HIP;
    weno_l2is_destroy(kv.second);
    kv.second = nullptr;
    ++n;
  }
  g_cache.clear();
  if (n && hipSetDevice(cur) != hipSuccess) return WL2_E_HIP;
  return n;
}

int weno_l2is_step(weno_l2is_ctx* c, double* U, double dt) {
  if (!c || !U) return WL2_E_NULL;
  if (dt > 0.0 && !std::isfinite(dt)) return WL2_E_PARAM;
  if (inflow_missing(c)) return WL2_E_BC;
  hipError_t e = launch_cfl(c, U, dt > 0.0 ? dt : 0.0, 0);
  if (e == hipSuccess) e = rk3(c, U);
  return hip_err(e);
}

int weno_l2is_advance(weno_l2is_ctx* c, double* U, int n_steps, double t_end) {
  if (!c || !U) return WL2_E_NULL;
  if (n_steps < 0 || !(t_end > 0.0) || !std::isfinite(t_end)) return WL2_E_PARAM;
  if (inflow_missing(c)) return WL2_E_BC;
  hipLaunchKernelGGL(set_t_end_kernel, dim3(1), dim3(64), 0, c->stream, c->ctl, t_end);
  hipError_t e = hipGetLastError();
  // small 1D grids: every step in one single-workgroup launch
  if (e == hipSuccess && use_row_steps(c)) {
    TimedLaunch tl(c, "row1d_steps");
    return hip_err(row1d_steps(U, c->U1, c->U2, c->ctl, c->list, c->p.cfl * c->dx, n_steps,
                               c->p.split == WL2_SPLIT_LLF && c->p.hybrid == WL2_HYB_PER_FIELD,
                               c->g, c->ph, c->stream));
  }
  // fused 3D and row 1D/2D paths: the last stage of a step also reduces the
  // CFL speed of the new state (its cells are in registers there), so every
  // step after the first of this call skips the separate reduction.  Within
  // one call U is only touched here, so the folded maximum is that of U.
  const bool fold = use_fused(c) || use_row(c);
  for (int s = 0; s < n_steps && e == hipSuccess; ++s) {
    // 1D/2D: from the second step the stage-1 kernel forms dt itself from
    // the folded maximum (one launch per step less)
    const bool kclock = s > 0 && use_row(c);
    if (!kclock) e = launch_cfl(c, U, 0.0, 1, fold && s > 0);
    if (e == hipSuccess) e = rk3(c, U, fold && s + 1 < n_steps, kclock);
  }
  return hip_err(e);
}

int weno_l2is_set_time(weno_l2is_ctx* c, double t) {
  if (!c) return WL2_E_NULL;
  if (!std::isfinite(t)) return WL2_E_PARAM;
  StepCtl h;
  hipError_t e = hipMemcpyAsync(&h, c->ctl, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return WL2_E_HIP;
  h.t = t;
  e = hipMemcpyAsync(c->ctl, &h, sizeof(h), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return hip_err(e);
}

int weno_l2is_cfl_dt(weno_l2is_ctx* c, const double* U, double* dt_host) {
  if (!c || !U) return WL2_E_NULL;
  hipError_t e = launch_cfl(c, U, 0.0, 0);
  if (e != hipSuccess) return WL2_E_HIP;
  if (!dt_host) return WL2_OK;
  StepCtl h;
  e = hipMemcpyAsync(&h, c->ctl, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return WL2_E_HIP;
  *dt_host = h.dt;
  return (h.status & 1u) ? WL2_S_NONPHYSICAL : WL2_OK;
}

int weno_l2is_time(weno_l2is_ctx* c, double* t_host, double* last_dt_host, unsigned* steps) {
  if (!c) return WL2_E_NULL;
  StepCtl h;
  hipError_t e = hipMemcpyAsync(&h, c->ctl, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return WL2_E_HIP;
  if (t_host) *t_host = h.t;
  if (last_dt_host) *last_dt_host = h.dt;
  if (steps) *steps = h.steps;
  return WL2_OK;
}

int weno_l2is_face_debug(weno_l2is_ctx* c, const double* U, int dir, unsigned char* flags,
                         double* sigma) {
  if (!c || !U || !flags || !sigma) return WL2_E_NULL;
  if (dir < 0 || dir >= c->dim) return WL2_E_PARAM;
  if (inflow_missing(c)) return WL2_E_BC;
  long long nface = c->ncell / c->n[dir] * (c->n[dir] + 1);
  const size_t nout = (size_t)c->nvar * (size_t)nface, ubytes = sizeof(double) * c->nvar * (size_t)c->ncell;
  if (overlaps(U, ubytes, flags, nout) || overlaps(U, ubytes, sigma, nout * sizeof(double)) ||
      overlaps(flags, nout, sigma, nout * sizeof(double)))
    return WL2_E_PARAM;
  const long long blocks = (nface + 255) / 256;
  if (blocks > 0x7fffffffLL) return WL2_E_SHAPE;
  const dim3 gr((unsigned)blocks), bl(256);
  if (fill_yghosts(c, U, -1.0) != hipSuccess) return WL2_E_HIP;
#define WL2_DBG(NV, D) \
  hipLaunchKernelGGL((face_debug_kernel<NV, D>), gr, bl, 0, c->stream, U, c->g, c->ph, flags, sigma, nface)
  switch (c->nvar * 3 + dir) {
    case 9: WL2_DBG(3, 0); break;
    case 12: WL2_DBG(4, 0); break;
    case 13: WL2_DBG(4, 1); break;
    case 15: WL2_DBG(5, 0); break;
    case 16: WL2_DBG(5, 1); break;
    case 17: WL2_DBG(5, 2); break;
    default: return WL2_E_PARAM;
  }
#undef WL2_DBG
  return hip_err(hipGetLastError());
}

int weno_l2is_status(weno_l2is_ctx* c, unsigned* status_bits, int clear) {
  if (!c) return WL2_E_NULL;
  StepCtl h;
  hipError_t e = hipMemcpyAsync(&h, c->ctl, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return WL2_E_HIP;
  if (status_bits) *status_bits = h.status;
  if (clear && h.status) {
    const unsigned zero = 0;
    e = hipMemcpyAsync(&c->ctl->status, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return WL2_E_HIP;
  }
  return h.status ? WL2_S_NONPHYSICAL : WL2_OK;
}

int weno_l2is_tune(weno_l2is_ctx* c, int path, int zchunk, int waves_per_simd) {
  if (!c) return WL2_E_NULL;
  if (path < WL2_PATH_AUTO || path > WL2_PATH_FUSED_CELLS || zchunk < 0) return WL2_E_PARAM;
  if (waves_per_simd < 0 || waves_per_simd > 2) return WL2_E_PARAM;

  c->path = path;
  c->zchunk = zchunk;
  c->wpe = waves_per_simd == 0 ? 2 : waves_per_simd;
  return WL2_OK;
}

int weno_l2is_timing_enable(weno_l2is_ctx* c, int enable) {
  if (!c) return WL2_E_NULL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return WL2_E_HIP;
  c->ev_used.clear();
  c->knames.clear();
  c->timing = enable != 0;
  return WL2_OK;
}

int weno_l2is_timing_read(weno_l2is_ctx* c, int cap, char* names, double* total_ms,
                          long long* launches, int* n_kernels) {
  if (!c || !n_kernels) return WL2_E_NULL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return WL2_E_HIP;
  const int nk = (int)c->knames.size();
  std::vector<double> tot(nk, 0.0);
  std::vector<long long> cnt(nk, 0);
  for (auto& u : c->ev_used) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_pool[u.second], c->ev_pool[u.second + 1]) != hipSuccess)
      return WL2_E_HIP;
    tot[u.first] += ms;
    cnt[u.first] += 1;
  }
  const int m = nk < cap ? nk : cap;
  for (int k = 0; k < m; ++k) {
    if (names) {
      std::strncpy(names + 64 * k, c->knames[k].c_str(), 63);
      names[64 * k + 63] = 0;
    }
    if (total_ms) total_ms[k] = tot[k];
    if (launches) launches[k] = cnt[k];
  }
  *n_kernels = m;
  return WL2_OK;
}

const char* weno_l2is_strerror(int code) {
  switch (code) {
    case WL2_OK: return "ok";
    case WL2_E_NULL: return "required pointer is NULL";
    case WL2_E_SHAPE: return "invalid grid shape";
    case WL2_E_PARAM: return "invalid parameter";
    case WL2_E_BC: return "invalid boundary conditions";
    case WL2_E_HIP: return "HIP runtime error";
    case WL2_E_NOMEM: return "device allocation failed";
    case WL2_E_BUDGET: return "HBM budget or slot table exhausted";
    case WL2_E_SLOT: return "slot not in use or not finished";
    case WL2_S_NONPHYSICAL: return "non-physical state detected";
  }
  return "unknown code";
}

}  // extern "C"
