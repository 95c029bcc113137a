// Fused 3D stage kernel (gfx950, FP64): all three sweep directions, the flux
// difference of Eq.(19) and the SSP-RK3 stage combination in one pass over
// HBM.
//
// Work decomposition.  A workgroup of 256 threads owns a 16 x 15 (x, y) tile
// of columns and marches along z through a chunk of planes.  Each of the 240
// column owners keeps a six-cell register window of "light" records
// (U, p, c, 1/sqrt(rho)) of its column, so every z face is computed from
// registers.  The current plane, with a three-cell halo in x and y, is staged
// in LDS; one thread per face computes the (16+1) x 15 = 255 x faces and the
// 16 x (15+1) = 256 y faces (two balanced rounds), and the face fluxes are
// exchanged through LDS so that every cell receives its six face fluxes from
// exactly one owner, in a fixed order (the result is deterministic).
// Physical fluxes along the face direction are formed on the fly from the
// light record.  Every face takes the linear branch here; a cell next to a
// face whose detector asks for the nonlinear flux is appended (with its
// face mask) to a correction list, and the face itself to the face list of
// its direction.  The correction kernels then compute each listed face's
// change (WENO-L2IS minus linear) once (weno_flist3d_kernel) and add the
// changes of each listed cell's faces in a fixed order
// (weno_sumlist3d_kernel); weno_fix3d_kernel is the per-cell form, which
// computes each face for both of its cells.
// Tiles are numbered so that the workgroups resident on one XCD (dispatch is
// round-robin over the 8 XCDs) take a contiguous range of tiles and share
// their halos in that XCD's L2.  A tile at the high x or y edge of the grid
// (256 = 17 x 15 + 1 rows leaves a last tile row one cell high) computes
// only the faces of its in-grid cells and loads only the records they read
// (whole wavefronts then skip the work).
#pragma once
#include "wl2_fused_launch.hpp"
#include "wl2_lface.hpp"

namespace wl2 {

constexpr int FT_THREADS = 256;
constexpr int FT_OWN = FT_X * FT_Y;              // 240 column owners
constexpr int FP_X = FT_X + 6, FP_Y = FT_Y + 6;  // LDS plane pitch (with halo)
// LDS plane layout: row-major cells, the eight record values of a row
// interleaved (row, value, column), so the 48 values of an x-face stencil
// lie within the immediate-offset reach of one LDS address (a y-face
// stencil within four) instead of one address per value plane.
// The row pitch is one double longer than the eight value rows: the odd
// pitch moves the rows that one LDS instruction of a wavefront touches
// (16-17 lanes per row) onto different banks.  Measured at 256^3: pitch
// +1 is 3 % faster than +0, +2, +3 or +4 (+4 is the largest that keeps two
// workgroups per CU).
constexpr int FP_ROW = 8 * FP_X + 1;  // doubles per LDS row (NV + 3 = 8 values)
constexpr int NXF = (FT_X + 1) * FT_Y;           // 255 x faces per plane
constexpr int NYF = FT_X * (FT_Y + 1);           // 256 y faces per plane
constexpr int NHALO = 6 * FT_Y + 6 * FT_X;       // 186 halo cells per plane

struct FusedArgs {
  const double* Uk;   // stage input
  double* out;        // RK: U^(k+1); RHS: dU/dt
  const double* Un;   // RK: U^n (read when rk_a != 0)
  const StepCtl* ctl;
  double rk_a, rk_b;
  int zc;             // planes per workgroup
  int tiles_x, tiles_y;
  unsigned long long* list;  // cells next to a face that needs the WENO flux
  unsigned int* list_n;      // entries listed in this stage (all workgroups; zero
                             // when the stage starts)
  unsigned int* list_clear;  // the next stage's counter, zeroed by the correction kernel
  unsigned int* counts;      // entries each workgroup listed in its list region
  unsigned int* offs;        // exclusive prefix sums of counts (nreg + 1 values)
  StepCtl* cfl;              // RK: if set, fold the CFL speed of the new state
                             // into cfl->smax / status (next step's dt)
  // face lists (or null: per-cell corrections): the faces that need the
  // WENO flux, the x, y and z lists back to back, each cut into one region
  // per workgroup as the cell list is.  An entry locates its face inside
  // the workgroup's tile: slot + 256 * (plane - z0), with slot = row * 17 +
  // fx for an x face (fx = 0 at the tile's x0 - 1/2), fy * 16 + col for a y
  // face and oy * 16 + ox for a z face, whose plane is the index of the face
  // (between cells plane - 1 and plane).
  unsigned int* flist;
  unsigned int* counts_f;    // faces each workgroup listed, [direction][region]
  unsigned int* offs_f;      // their exclusive prefix sums over (direction, region)
  double* D;                 // face changes of the listed faces: x, y, z faces, 5
                             // values each, [face][v] (a face's values together:
                             // the lists visit faces in no spatial order)
};

// The correction list is cut into one region per workgroup of the stage
// kernel, so that no global counter is shared: the regions of all
// workgroups tile [0, ncell) in logical tile order, each as large as the
// workgroup's in-grid cells (only the last tile along x, the last tile row
// and the last z chunk are partial, so every region before a given one is
// full-sized).  First list index of the region of logical tile r.
// Regions up to which a correction kernel keeps the list offsets in LDS
// (the per-cell kernel forms them there itself; beyond, a one-workgroup scan
// kernel writes them to global memory, as it always does for face lists).
constexpr int SCAN_LDS = 8192;

__device__ __forceinline__ long long list_region_start(const FusedArgs& a, const KGrid& g, int r) {
  const int ttx = r % a.tiles_x, rest = r / a.tiles_x;
  const int tty = rest % a.tiles_y, tzc = rest / a.tiles_y;
  const long long z0 = (long long)tzc * a.zc;
  const long long planes = min((long long)a.zc, (long long)g.n[2] - z0);
  const long long vr = min(FT_Y, g.n[1] - tty * FT_Y);
  return (long long)g.n[0] * g.n[1] * z0 +
         ((long long)tty * FT_Y * g.n[0] + (long long)ttx * FT_X * vr) * planes;
}

// First index of the face-list region of direction d of logical tile r,
// counted from the start of the x list.  Each workgroup lists the faces it
// owns: along x the faces x0 .. x0 + cols - 1 of each of its rows, and in
// the last tile along x also the last face of the row; along y alike; along
// z the faces z0 + 1 .. z1 of each column, and in the first z chunk also
// face 0.  So the regions of a direction tile [0, faces of that direction)
// in logical tile order, and every region before a given one is full-sized
// where it matters (as for the cell list).
__device__ __forceinline__ long long flist_region_start(const FusedArgs& a, const KGrid& g, int d,
                                                        int r) {
  const int ttx = r % a.tiles_x, rest = r / a.tiles_x;
  const int tty = rest % a.tiles_y, tzc = rest / a.tiles_y;
  const long long nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long z0 = (long long)tzc * a.zc;
  const long long planes = min((long long)a.zc, nz - z0);
  const long long rows = min((long long)FT_Y, ny - (long long)tty * FT_Y);
  if (d == 0)
    return (nx + 1) * ny * z0 + ((long long)tty * FT_Y * (nx + 1) + (long long)ttx * FT_X * rows) * planes;
  const long long nfx = (nx + 1) * ny * nz;
  if (d == 1) {
    const long long rowsy = rows + (tty == a.tiles_y - 1 ? 1 : 0);
    return nfx + nx * (ny + 1) * z0 + ((long long)tty * FT_Y * nx + (long long)ttx * FT_X * rowsy) * planes;
  }
  const long long nfy = nx * (ny + 1) * nz;
  const long long planesz = planes + (tzc == 0 ? 1 : 0);
  return nfx + nfy + nx * ny * (z0 + (tzc > 0 ? 1 : 0)) +
         ((long long)tty * FT_Y * nx + (long long)ttx * FT_X * rows) * planesz;
}

// The faces of the owner's cell (ox, oy, plane z0 + pl) flagged in its mask
// m (x-, x+, y-, y+, z-, z+) that this workgroup lists: every flagged face
// below the cell along x and y, the one above along z, and the faces above
// along x (y) in the last tile along x (y) and below along z in plane 0,
// which no other cell of a workgroup lists.  Entries as in FusedArgs::flist.
__device__ __forceinline__ void list_faces(const FusedArgs& a, unsigned int* const (&fl)[3],
                                           unsigned int* cnt, unsigned m, int t, int ox, int oy, int pl,
                                           bool plane0, bool last_x, bool last_y) {
  const unsigned int p = 256u * (unsigned)pl;
  const unsigned int sx = (unsigned)(oy * (FT_X + 1) + ox);
  if (m & 1u) fl[0][atomicAdd(&cnt[0], 1u)] = sx + p;
  if ((m & 2u) && last_x) fl[0][atomicAdd(&cnt[0], 1u)] = sx + 1u + p;
  if (m & 4u) fl[1][atomicAdd(&cnt[1], 1u)] = (unsigned)t + p;
  if ((m & 8u) && last_y) fl[1][atomicAdd(&cnt[1], 1u)] = (unsigned)(t + FT_X) + p;
  if (m & 32u) fl[2][atomicAdd(&cnt[2], 1u)] = (unsigned)t + p + 256u;
  if ((m & 16u) && plane0) fl[2][atomicAdd(&cnt[2], 1u)] = (unsigned)t;
}

typedef __attribute__((address_space(3))) double lds_wdouble;
typedef const __attribute__((address_space(3))) double lds_double;

// The LDS address of p, opaque to the compiler so that it is not split into
// a register part and a constant too large for an instruction offset (the
// offsets of the values around it then fold into the LDS instructions).
__device__ __forceinline__ lds_wdouble* lds_addr(double* p) {
  lds_wdouble* q = (lds_wdouble*)p;
  asm volatile("" : "+v"(q));
  return q;
}

template <int NV>
__device__ __forceinline__ void lds_put(double* srec, int idx, const LRec<NV>& r) {
  static_assert(NV + 3 == 8, "eight values per LDS cell");
  lds_wdouble* q = lds_addr(srec + idx);
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v * FP_X] = r.U[v];
  q[NV * FP_X] = r.p;
  q[(NV + 1) * FP_X] = r.c;
  q[(NV + 2) * FP_X] = r.iw;
}

// z-window ring of a column owner: the eight values of a record as four
// pairs, each an aligned 16-byte LDS word per owner (one 128-bit access
// per pair, consecutive owners at consecutive words).
constexpr int RING_SLOT = 4 * FT_OWN;  // double2 words per ring slot

template <int NV>
__device__ __forceinline__ void ring_store(double2* swin, int slot, int t, const LRec<NV>& r) {
  static_assert(NV == 5, "five conserved values: four pairs per record");
  double2* q = swin + slot * RING_SLOT + t;
  q[0] = make_double2(r.U[0], r.U[1]);
  q[FT_OWN] = make_double2(r.U[2], r.U[3]);
  q[2 * FT_OWN] = make_double2(r.U[4], r.p);
  q[3 * FT_OWN] = make_double2(r.c, r.iw);
}

template <int NV>
__device__ __forceinline__ void ring_load(const double2* swin, int slot, int t, LRec<NV>& r) {
  const double2* q = swin + slot * RING_SLOT + t;
  const double2 a = q[0], b = q[FT_OWN], c = q[2 * FT_OWN], d = q[3 * FT_OWN];
  r.U[0] = a.x;
  r.U[1] = a.y;
  r.U[2] = b.x;
  r.U[3] = b.y;
  r.U[4] = c.x;
  r.p = c.y;
  r.c = d.x;
  r.iw = d.y;
}

// Stencil accessor over the LDS plane: six cells at p + m * stride, p an
// opaque LDS address (lds_addr).
template <int NV>
struct LdsSrc {
  const lds_double* p;
  int stride;
  __device__ __forceinline__ void get(int m, LRec<NV>& r) const {
    const lds_double* q = p + m * stride;
#pragma unroll
    for (int v = 0; v < NV; ++v) r.U[v] = q[v * FP_X];
    r.p = q[NV * FP_X];
    r.c = q[(NV + 1) * FP_X];
    r.iw = q[(NV + 2) * FP_X];
  }
};

// The LDS address of srec[idx], opaque to the compiler so that it is not
// split into a register part and a constant too large for an instruction
// offset.
__device__ __forceinline__ const lds_double* lds_addr(const double* srec, int idx) {
  const lds_double* p = (const lds_double*)(srec + idx);
  asm volatile("" : "+v"(p));
  return p;
}

// Column of cells at fixed (x, y): element offset of its (x, y) position
// after the boundary mapping, and the momentum signs of mirror ghosts.
struct Col {
  long long xy;
  bool fx, fy;
};

__device__ __forceinline__ Col make_col(const KGrid& g, int x, int y) {
  Col c;
  const int ix = ghost_clamped(x, g.n[0], g.bc_lo[0], g.bc_hi[0], c.fx);
  const int iy = ghost_clamped(y, g.n[1], g.bc_lo[1], g.bc_hi[1], c.fy);
  c.xy = ix + (long long)iy * g.stride[1];
  return c;
}

// Cell z of a column, as stored (a reflective ghost is the mirror cell; its
// normal momentum is negated by col_flip when the value is used, so that a
// prefetch does not have to wait for the load).
template <int NV>
__device__ __forceinline__ void load_col_raw(const double* __restrict__ U, const KGrid& g,
                                             const Col& c, int z, double (&u)[NV]) {
  bool fz = false;
  const int iz = (z >= 0 && z < g.n[2]) ? z : ghost_clamped(z, g.n[2], g.bc_lo[2], g.bc_hi[2], fz);
  const long long off = c.xy + (long long)iz * g.stride[2];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = U[v * g.ncell + off];
}

template <int NV>
__device__ __forceinline__ void col_flip(const KGrid& g, const Col& c, int z, double (&u)[NV]) {
  bool fz = false;
  if (z < 0 || z >= g.n[2]) (void)ghost_clamped(z, g.n[2], g.bc_lo[2], g.bc_hi[2], fz);
  if (c.fx) u[1] = -u[1];
  if (c.fy) u[2] = -u[2];
  if (fz) u[3] = -u[3];
}

template <int NV>
__device__ __forceinline__ void load_col(const double* __restrict__ U, const KGrid& g, const Col& c,
                                         int z, double (&u)[NV]) {
  load_col_raw<NV>(U, g, c, z, u);
  col_flip<NV>(g, c, z, u);
}

// z stencil of a column owner: cells j-2, j-1 from the per-column LDS ring,
// j .. j+3 from registers.
template <int NV>
struct ZSrc {
  const double2* swin;
  int slot0, slot1, col;
  const LRec<NV>&r0, &r1, &r2, &r3;
  __device__ __forceinline__ void get(int m, LRec<NV>& r) const {
    if (m == 0) ring_load<NV>(swin, slot0, col, r);
    else if (m == 1) ring_load<NV>(swin, slot1, col, r);
    else r = m == 2 ? r0 : m == 3 ? r1 : m == 4 ? r2 : r3;
  }
};

// WPE: target waves per SIMD.  SPLIT / HYB: compile-time modes (-1: runtime).
template <int OUT, int WPE, int SPLIT, int HYB>
__global__ __launch_bounds__(FT_THREADS, WPE) void fused3d_kernel(FusedArgs a, KGrid g, KPhys ph) {
  constexpr int NV = 5;
  __shared__ double srec[FP_Y * FP_ROW];     // plane z with halo (row, value, column)
  __shared__ double sfx[NV][NXF];            // x-face fluxes of plane z
  __shared__ double sfy[NV][NYF];            // y-face fluxes of plane z
  __shared__ double2 swin[2 * RING_SLOT];    // two oldest cells of each z window
  __shared__ unsigned char sgx[NXF], sgy[NYF];  // face needs the nonlinear flux
  __shared__ unsigned char scm[FT_OWN];          // face mask of the owner's last cell
  __shared__ unsigned int s_cnt;                 // entries listed by this workgroup
  __shared__ unsigned int s_fcnt[3];             // faces listed per direction
  __shared__ unsigned int s_any[2];              // plane z - 1 has faces to list: s_any[z & 1]

  double dt = 0.0;
  if (OUT == OUT_RK) {
    dt = a.ctl->dt;
    if (!(dt > 0.0)) return;  // uniform across the grid: finished run
  }
  const unsigned long long* lfx = a.ctl->lf_bits[0];  // read only for LF splitting
  const unsigned long long* lfy = a.ctl->lf_bits[1];
  const unsigned long long* lfz = a.ctl->lf_bits[2];

  // XCD-aware tile order: the blocks dispatched to one XCD (b mod 8) get a
  // contiguous range of logical tile ids.
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb / 8, r8 = nb % 8, xcd = b % 8, j = b / 8;
  const int logical = (xcd < r8 ? xcd * (q + 1) : r8 * (q + 1) + (xcd - r8) * q) + j;
  const int ttx = logical % a.tiles_x;
  const int rest = logical / a.tiles_x;
  const int tty = rest % a.tiles_y;
  const int tzc = rest / a.tiles_y;
  const int x0 = ttx * FT_X, y0 = tty * FT_Y;
  const int z0 = tzc * a.zc;
  const int z1 = min(z0 + a.zc, g.n[2]);

  const int t = threadIdx.x;
  const bool owner = t < FT_OWN;
  const int ox = t % FT_X, oy = t / FT_X;
  const int gx = x0 + ox, gy = y0 + oy;
  const bool valid = owner && gx < g.n[0] && gy < g.n[1];
  // extent of the tile inside the grid (smaller in the tiles at the high x
  // and y edges): only the faces of in-grid cells are computed
  const int cols_v = min(FT_X, g.n[0] - x0), rows_v = min(FT_Y, g.n[1] - y0);
  const int lds_own = (oy + 3) * FP_ROW + (ox + 3);
  const Col ocol = make_col(g, gx, gy);
  const long long oout = (long long)gx + (long long)gy * g.stride[1];
  // this workgroup's region of the correction list (its count is kept in
  // LDS and stored at the end; made visible by the barriers of the first
  // plane before any append)
  const long long reg0 = list_region_start(a, g, logical);
  // face lists: this workgroup's region of each direction's list
  const bool flists = HYB != HYB_WENO_ONLY && HYB != HYB_LINEAR_ONLY && a.flist != nullptr;
  unsigned int* fl[3] = {nullptr, nullptr, nullptr};
  if (flists) {
#pragma unroll
    for (int d = 0; d < 3; ++d) fl[d] = a.flist + flist_region_start(a, g, d, logical);
  }
  if (t == 0) {
    s_cnt = 0u;
    s_fcnt[0] = 0u;
    s_fcnt[1] = 0u;
    s_fcnt[2] = 0u;
    s_any[0] = 0u;
    s_any[1] = 0u;
  }

  // halo cell of this thread (t < NHALO): tile-relative (hc, hr)
  int hc = 0, hr = 0;
  if (t < 6 * FT_Y) {
    hr = t / 6;
    const int k = t % 6;
    hc = k < 3 ? k - 3 : FT_X + k - 3;
  } else if (t < NHALO) {
    const int h = t - 6 * FT_Y;
    hc = h % FT_X;
    const int k = h / FT_X;
    hr = k < 3 ? k - 3 : FT_Y + k - 3;
  }
  const int lds_halo = (hr + 3) * FP_ROW + (hc + 3);
  const Col hcol = make_col(g, x0 + hc, y0 + hr);
  // records that a computed face reads: tile columns up to cols_v + 2 and
  // rows up to rows_v + 2 (all of them except in the edge tiles)
  const bool own_need = owner && ox < cols_v + 3 && oy < rows_v + 3;
  const bool halo_need = t < NHALO && hc < cols_v + 3 && hr < rows_v + 3;

  // owner registers: r0..r3 = cells z-1 .. z+2 at the top of iteration z;
  // the ring holds cell c in slot (c & 1)
  LRec<NV> r0, r1, r2, r3;
  double Fzp[NV];
  bool zprev = false;  // face z - 1/2 needs the nonlinear flux
  double upre[NV], hpre[NV];
  double cfl_max = 0.0;  // CFL speed of the cells written here (a.cfl set)
  bool cfl_bad = false;
  double unp[NV] = {};  // U^n of cell z (RK stages 2, 3), loaded a phase ahead
  if (own_need) {
    double u[NV];
    LRec<NV> c0, c1;
    load_col<NV>(a.Uk, g, ocol, z0 - 3, u);
    make_lrec<NV>(u, ph, c0);
    load_col<NV>(a.Uk, g, ocol, z0 - 2, u);
    make_lrec<NV>(u, ph, c1);
    load_col<NV>(a.Uk, g, ocol, z0 - 1, u);
    make_lrec<NV>(u, ph, r0);
    load_col<NV>(a.Uk, g, ocol, z0, u);
    make_lrec<NV>(u, ph, r1);
    load_col<NV>(a.Uk, g, ocol, z0 + 1, u);
    make_lrec<NV>(u, ph, r2);
    load_col<NV>(a.Uk, g, ocol, z0 + 2, u);
    make_lrec<NV>(u, ph, r3);
    // ring: cells z0-3 and z0-2
    const int s3 = (z0 - 3) & 1, s2 = (z0 - 2) & 1;
    ring_store<NV>(swin, s3, t, c0);
    ring_store<NV>(swin, s2, t, c1);
    // face z0 - 1/2 (cells z0-3 .. z0+2): window c0, c1, r0, r1, r2, r3
    const WinSrc<NV> src{c0, c1, r0, r1, r2, r3};
    zprev = face_linear_l<NV, 2, SPLIT, HYB>(src, ph, ph.eps_thr[2], lfz, Fzp) != 0u;
    load_col_raw<NV>(a.Uk, g, ocol, z0 + 3, upre);
  }
  if (halo_need) load_col_raw<NV>(a.Uk, g, hcol, z0, hpre);

  for (int z = z0; z < z1; ++z) {
    if (own_need) {
      // retire cell z-1 into the ring (overwrites cell z-3), then shift:
      // registers become cells z .. z+3
      const int sl = (z - 1) & 1;
      ring_store<NV>(swin, sl, t, r0);
      r0 = r1;
      r1 = r2;
      r2 = r3;
      col_flip<NV>(g, ocol, z + 3, upre);
      make_lrec<NV>(upre, ph, r3);
      lds_put<NV>(srec, lds_own, r0);  // cell z
      // The prefetch of cell z+4 lands in the registers just consumed.  The
      // empty asm (a compiler memory barrier that takes the new record as
      // input) keeps the loads below the last use of the old values: loads
      // hoisted above it need other registers and a copy, and the copy waits
      // for the load.  The load is unconditional (past the chunk the index is
      // ghost-clamped and stays in bounds) for the same reason.
      asm volatile("" ::"v"(r3.U[0]), "v"(r3.U[1]), "v"(r3.U[2]), "v"(r3.U[3]), "v"(r3.U[4]),
                   "v"(r3.p), "v"(r3.c), "v"(r3.iw)
                   : "memory");
      load_col_raw<NV>(a.Uk, g, ocol, z + 4, upre);
      if (OUT == OUT_RK && a.rk_a != 0.0) {
        // U^n and the output are streamed once (non-temporal), leaving L2 to
        // the stage input, whose cells are also halo of the neighbour tiles.
        // Clamped column (equal to the cell's own index for valid owners).
        const long long offn = ocol.xy + (long long)z * g.stride[2];
#pragma unroll
        for (int v = 0; v < NV; ++v) unp[v] = __builtin_nontemporal_load(&a.Un[v * g.ncell + offn]);
      }
    }
    if (halo_need) {
      LRec<NV> hrec;
      col_flip<NV>(g, hcol, z, hpre);
      make_lrec<NV>(hpre, ph, hrec);
      lds_put<NV>(srec, lds_halo, hrec);
      asm volatile("" ::: "memory");  // as above: the prefetch after the last use
      load_col_raw<NV>(a.Uk, g, hcol, z + 1, hpre);
    }
    __syncthreads();
    // the next plane's flag starts clear (its last reader, the previous
    // plane's append point, is behind this barrier; its first writer comes
    // after this plane's second one)
    if (flists && t == 0) s_any[(z + 1) & 1] = 0u;
    __builtin_amdgcn_s_setprio(0);  // face rounds at normal priority
    __builtin_amdgcn_sched_barrier(0);
    // x faces: thread t < 255 -> row t/17, face fx = t%17 at x0 + fx - 1/2
    if (t < NXF && t / (FT_X + 1) < rows_v && t % (FT_X + 1) <= cols_v) {
      const int row = t / (FT_X + 1), fx = t % (FT_X + 1);
      const LdsSrc<NV> src{lds_addr(srec, (row + 3) * FP_ROW + fx), 1};
      double F[NV];
      sgx[t] = face_linear_l<NV, 0, SPLIT, HYB>(src, ph, ph.eps_thr[0], lfx, F) != 0u;
#pragma unroll
      for (int v = 0; v < NV; ++v) sfx[v][t] = F[v];
    }
    __builtin_amdgcn_sched_barrier(0);
    // y faces: thread t -> column t%16, face fy = t/16 at y0 + fy - 1/2
    if (t % FT_X < cols_v && t / FT_X <= rows_v) {
      const int col = t % FT_X, fy = t / FT_X;
      const LdsSrc<NV> src{lds_addr(srec, fy * FP_ROW + col + 3), FP_ROW};
      double F[NV];
      sgy[t] = face_linear_l<NV, 1, SPLIT, HYB>(src, ph, ph.eps_thr[1], lfy, F) != 0u;
#pragma unroll
      for (int v = 0; v < NV; ++v) sfy[v][t] = F[v];
    }
    __syncthreads();
    // raised wave priority from here (z face, stores, the next plane's loads
    // and records) to the next plane's first barrier: the waves that issue
    // memory requests go before the other workgroup's face rounds (measured
    // 1.2-1.7 % faster at 256^3; a wave's priority is local to this kernel)
    __builtin_amdgcn_s_setprio(2);
    __builtin_amdgcn_sched_barrier(0);
    if (flists && z > z0 && s_any[z & 1]) {
      // the faces of the previous plane's cells that need the WENO flux go
      // to the face lists (from the cell masks kept in LDS, here where few
      // registers are live; only in planes where some cell had a mask)
      if (valid) list_faces(a, fl, s_fcnt, scm[t], t, ox, oy, z - 1 - z0, z - 1 == 0,
                            ox == cols_v - 1 && ttx == a.tiles_x - 1,
                            oy == rows_v - 1 && tty == a.tiles_y - 1);
    }
    if (valid) {
      // z face z + 1/2: cells z-2, z-1 (ring), z .. z+3 (registers)
      double Fz[NV];
      const ZSrc<NV> src{swin, (z - 2) & 1, (z - 1) & 1, t, r0, r1, r2, r3};
      const bool zcur = face_linear_l<NV, 2, SPLIT, HYB>(src, ph, ph.eps_thr[2], lfz, Fz) != 0u;
      const int ix = oy * (FT_X + 1) + ox;
      const int iy = oy * FT_X + ox;
      const long long off = oout + (long long)z * g.stride[2];
      // faces of this cell that need the nonlinear flux: x-, x+, y-, y+, z-, z+
      unsigned cm = 0;
      if (valid) {
        cm = (sgx[ix] ? 1u : 0u) | (sgx[ix + 1] ? 2u : 0u) | (sgy[iy] ? 4u : 0u) |
             (sgy[iy + FT_X] ? 8u : 0u) | (zprev ? 16u : 0u) | (zcur ? 32u : 0u);
      }
      zprev = zcur;
      // wave-aggregated append to the correction list (none when every
      // face is WENO by construction: the correction kernel then walks all
      // cells)
      if (HYB != HYB_WENO_ONLY) {
        const unsigned long long ball = __ballot(cm != 0u);
        if (ball) {
          const int lane = threadIdx.x & 63;
          const int leader = __ffsll((long long)ball) - 1;
          unsigned int basei = 0;
          if (lane == leader) {
            basei = atomicAdd(&s_cnt, (unsigned int)__popcll(ball));
            if (flists) s_any[(z + 1) & 1] = 1u;
          }
          basei = __shfl(basei, leader, 64);
          if (cm) {
            const unsigned int rank = __popcll(ball & ((1ull << lane) - 1ull));
            a.list[reg0 + basei + rank] = ((unsigned long long)off << 8) | cm;
          }
        }
      }
      if (valid) {
        double un[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double dU = ((sfx[v][ix] - sfx[v][ix + 1]) + (sfy[v][iy] - sfy[v][iy + FT_X]) +
                             (Fzp[v] - Fz[v])) * ph.inv_dx;
          if (OUT == OUT_RK) {
            double r = a.rk_b * (r0.U[v] + dt * dU);
            if (a.rk_a != 0.0) r += a.rk_a * unp[v];
            __builtin_nontemporal_store(r, &a.out[v * g.ncell + off]);
            un[v] = r;
          } else {
            __builtin_nontemporal_store(dU, &a.out[v * g.ncell + off]);
          }
        }
        // CFL speed of the new state; a listed cell is finished (and
        // counted) by the correction kernel
        if (OUT == OUT_RK && a.cfl != nullptr && cm == 0u) {
          const double m[3] = {un[1], un[2], un[3]};
          cfl_max = nan_max(cfl_max, cfl_speed<3>(un[0], m, un[4], ph.gamma, cfl_bad));
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Fzp[v] = Fz[v];
      // the z faces of the cell (bit 0: z - 1/2, bit 1: z + 1/2), listed at
      // the next plane's append point (kept in LDS, not in registers)
      if (flists) scm[t] = (unsigned char)cm;
    }
  }
  if (HYB != HYB_WENO_ONLY) {
    if (flists && z1 > z0) {
      __syncthreads();  // the last plane's masks and flag
      if (valid && s_any[z1 & 1])
        list_faces(a, fl, s_fcnt, scm[t], t, ox, oy, z1 - 1 - z0, z1 - 1 == 0,
                   ox == cols_v - 1 && ttx == a.tiles_x - 1, oy == rows_v - 1 && tty == a.tiles_y - 1);
    }
    __syncthreads();  // every append of the workgroup is counted
    if (t == 0) {
      a.counts[logical] = s_cnt;
      // the stage's total (zero at the stage's start): the correction
      // kernels return at once when nothing was listed
      if (s_cnt != 0u) atomicAdd(a.list_n, s_cnt);
    }
    if (flists && t < 3) a.counts_f[t * (int)gridDim.x + logical] = s_fcnt[t];
  }
  if (OUT == OUT_RK && a.cfl != nullptr) cfl_commit_wave(a.cfl, cfl_max, cfl_bad);
}

// Exclusive prefix sums of counts[0 .. n) into soffs[0 .. n] (LDS), by one
// block: each thread sums a contiguous run, the run sums are scanned
// (Hillis-Steele over at most 256 threads), then each run is written.
__device__ __forceinline__ void block_offsets(const unsigned int* counts, int n, unsigned int* soffs,
                                              unsigned int* spart) {
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int b = t * per, e = min(b + per, n);
  unsigned int sum = 0u;
  for (int r = b; r < e; ++r) sum += counts[r];
  spart[t] = sum;
  __syncthreads();
  for (int d = 1; d < nt; d <<= 1) {
    const unsigned int v = t >= d ? spart[t - d] : 0u;
    __syncthreads();
    spart[t] += v;
    __syncthreads();
  }
  unsigned int run = t > 0 ? spart[t - 1] : 0u;
  for (int r = b; r < e; ++r) {
    soffs[r] = run;
    run += counts[r];
  }
  if (t == nt - 1) soffs[n] = spart[nt - 1];
  __syncthreads();
}

// Index of the segment holding entry i: offs[lo] <= i < offs[lo + 1].
__device__ __forceinline__ int find_segment(const unsigned int* offs, int nseg, unsigned int i) {
  int lo = 0, hi = nseg;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offs[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The list offsets (nseg + 1 values written by list_scan_kernel) where a
// kernel looks them up: in global memory (L2) when no lane takes more than
// one of the n entries, else copied into LDS once per block (up to
// SCAN_LDS segments), so that the bisection of each entry runs in LDS.
__device__ __forceinline__ const unsigned int* stage_offsets(const unsigned int* offs, int nseg,
                                                             unsigned int n, unsigned int* soffs) {
  if (n <= gridDim.x * blockDim.x || nseg > SCAN_LDS) return offs;
  for (int r = threadIdx.x; r <= nseg; r += blockDim.x) soffs[r] = offs[r];
  __syncthreads();
  return soffs;
}

// Per listed cell: add the nonlinear part of the flux of its flagged faces,
// summed in the fixed order x-, x+, y-, y+, z-, z+, to the output (scaled by
// rk_b dt for a stage, 1 for dU/dt); eight lanes per cell (one per face) for
// a short list, one lane per cell for a long one, with the same bits.  Each
// cell is owned by one lane (group), so the result does not depend on
// scheduling.  With a.cfl set, the CFL speed of the corrected cell is folded.
// Two waves per SIMD (at most 256 registers; the default scheme's build
// spills 104 bytes): the stencil loads of a face are latency-bound, and at
// 256^3 two waves beat one by 16 % once shocklets form (3.18 against 3.78
// ms per step at 2.9 % WENO face-fields) and by 4 % in the smooth regime.
// W: the weighting of the reconstruction fixed at compile time (W_*), or -1
// to read it at run time.
template <int OUT, int SPLIT, int HYB, int W>
__global__ __launch_bounds__(128, 2) void weno_fix3d_kernel(FusedArgs a, KGrid g, KPhys ph) {
  constexpr int NV = 5;
  constexpr int GRP = 8;
  // the next stage's list starts empty (no kernel of this stage uses it)
  if (a.list_clear != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.list_clear = 0u;
  double scale = 1.0;
  if (OUT == OUT_RK) {
    const double dt = a.ctl->dt;
    if (!(dt > 0.0)) return;
    scale = a.rk_b * dt;
  }
  double cfl_max = 0.0;
  bool cfl_bad = false;
  // one listed cell (entry e): eight lanes of a group when grouped, else one lane
  auto fix_one = [&](unsigned long long e, bool grouped) {
    const long long off = (long long)(e >> 8);
    const unsigned cm = (unsigned)(e & 0xffu);
    const int x = (int)(off % g.n[0]);
    const int y = (int)((off / g.n[0]) % g.n[1]);
    const int z = (int)(off / g.stride[2]);
    double acc[NV];
    if (grouped) grouped_correction<NV, GRP, SPLIT, HYB, W>(a.Uk, g, ph, a.ctl, x, y, z, cm, acc);
    else serial_correction<NV, SPLIT, HYB, W>(a.Uk, g, ph, a.ctl, x, y, z, cm, acc);
    if (!grouped || (threadIdx.x % GRP) == 0) {
      double un[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        un[v] = a.out[v * g.ncell + off] + scale * (acc[v] * ph.inv_dx);
        a.out[v * g.ncell + off] = un[v];
      }
      if (OUT == OUT_RK && a.cfl != nullptr) {
        const double m[3] = {un[1], un[2], un[3]};
        cfl_max = nan_max(cfl_max, cfl_speed<3>(un[0], m, un[4], ph.gamma, cfl_bad));
      }
    }
  };
  if (HYB == HYB_WENO_ONLY) {
    // every face WENO (compile-time): every in-grid cell has all six faces
    // flagged, so the cells are walked in index order instead of a list (the
    // same cells and masks a list would hold; each cell's result does not
    // depend on the order)
    const unsigned int n = (unsigned int)g.ncell;
    const unsigned int threads = gridDim.x * blockDim.x;
    const unsigned int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const bool grouped = n <= threads / GRP;
    const unsigned int step = grouped ? threads / GRP : threads;
    for (unsigned int i = grouped ? tid / GRP : tid; i < n; i += step)
      fix_one(((unsigned long long)i << 8) | 0x3full, grouped);
  } else if (*a.list_n != 0u) {
    // the entries of all list regions as one index space: entry i lies in
    // the region r with offs[r] <= i < offs[r + 1], found by bisection.  Up
    // to SCAN_LDS regions every block forms the offsets in LDS from the
    // counts; beyond, list_scan_kernel has written them to a.offs.
    const int nreg = a.tiles_x * a.tiles_y * ((g.n[2] + a.zc - 1) / a.zc);
    __shared__ unsigned int soffs[SCAN_LDS + 1];
    __shared__ unsigned int spart[128];
    const unsigned int* offs = a.offs;
    if (nreg <= SCAN_LDS) {
      block_offsets(a.counts, nreg, soffs, spart);
      offs = soffs;
    }
    const unsigned int n = offs[nreg];
    const unsigned int threads = gridDim.x * blockDim.x;
    const unsigned int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const bool grouped = n <= threads / GRP;
    const unsigned int step = grouped ? threads / GRP : threads;
    for (unsigned int i = grouped ? tid / GRP : tid; i < n; i += step) {
      const int lo = find_segment(offs, nreg, i);
      fix_one(a.list[list_region_start(a, g, lo) + (i - offs[lo])], grouped);
    }
  }
  if (OUT == OUT_RK && a.cfl != nullptr) cfl_commit_wave(a.cfl, cfl_max, cfl_bad);
}

// Face lists, face-once corrections: every entry of the three face lists
// (taken as one index space over (direction, region), the offsets written by
// list_scan2_kernel) gives one face, whose change of flux (WENO
// minus linear, Eq.(20)-(28), (33)) goes to D[face][v] of its direction.
// One face per lane, and the lanes of a wavefront take consecutive entries,
// so that a wavefront runs faces of one direction (except where the x list
// meets the y list and the y list the z list).  The change depends on the
// face only: the same bits as weno_fix3d_kernel computes for either cell.
// W: the weighting of the reconstruction fixed at compile time (W_*), or -1
// to read it at run time.
template <int OUT, int SPLIT, int HYB, int W>
__global__ __launch_bounds__(128, 2) void weno_flist3d_kernel(FusedArgs a, KGrid g, KPhys ph) {
  constexpr int NV = 5;
  if (OUT == OUT_RK && !(a.ctl->dt > 0.0)) return;
  if (*a.list_n == 0u) return;  // no cell listed in this stage
  const int nreg = a.tiles_x * a.tiles_y * ((g.n[2] + a.zc - 1) / a.zc);
  const int nseg = 3 * nreg;
  __shared__ unsigned int soffs[SCAN_LDS + 1];
  const unsigned int n = a.offs_f[nseg];
  const unsigned int* offs = stage_offsets(a.offs_f, nseg, n, soffs);
  const long long nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long nfx = (nx + 1) * ny * nz, nfy = nx * (ny + 1) * nz;
  const unsigned int threads = gridDim.x * blockDim.x;
  for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += threads) {
    const int seg = find_segment(offs, nseg, i);
    const int d = seg / nreg, r = seg - d * nreg;
    const unsigned int e = a.flist[flist_region_start(a, g, d, r) + (i - offs[seg])];
    // the face from the tile of region r and the entry's slot and plane
    const int ttx = r % a.tiles_x, rest = r / a.tiles_x;
    const int tty = rest % a.tiles_y, tzc = rest / a.tiles_y;
    const int slot = (int)(e & 255u);
    const int z = tzc * a.zc + (int)(e >> 8);
    const int w = d == 0 ? FT_X + 1 : FT_X;
    const int x = ttx * FT_X + slot % w;
    const int y = tty * FT_Y + slot / w;
    const long long ex = nx + (d == 0), ey = ny + (d == 1);
    const long long f = x + ex * (y + ey * (long long)z);
    double dF[NV];
    double* D;
    if (d == 0) {
      face_delta<NV, 0, SPLIT, HYB, W>(a.Uk, g, ph, a.ctl->lf_bits[0], x, y, z, 0, dF);
      D = a.D;
    } else if (d == 1) {
      face_delta<NV, 1, SPLIT, HYB, W>(a.Uk, g, ph, a.ctl->lf_bits[1], x, y, z, 0, dF);
      D = a.D + NV * nfx;
    } else {
      face_delta<NV, 2, SPLIT, HYB, W>(a.Uk, g, ph, a.ctl->lf_bits[2], x, y, z, 0, dF);
      D = a.D + NV * (nfx + nfy);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) D[NV * f + v] = dF[v];
  }
}

// Face lists, per listed cell: the changes of its flagged faces read from D
// ([face][v]) and summed in the fixed order x-, x+, y-, y+, z-, z+ (+ below, - above),
// then added to the output exactly as weno_fix3d_kernel adds them (the same
// bits); with a.cfl set the CFL speed of the corrected cell is folded; the
// next stage's list counter is cleared.
template <int OUT>
__global__ __launch_bounds__(256) void weno_sumlist3d_kernel(FusedArgs a, KGrid g, KPhys ph) {
  constexpr int NV = 5;
  if (a.list_clear != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.list_clear = 0u;
  double scale = 1.0;
  if (OUT == OUT_RK) {
    const double dt = a.ctl->dt;
    if (!(dt > 0.0)) return;
    scale = a.rk_b * dt;
  }
  if (*a.list_n == 0u) return;  // no cell listed in this stage
  const int nreg = a.tiles_x * a.tiles_y * ((g.n[2] + a.zc - 1) / a.zc);
  __shared__ unsigned int soffs[SCAN_LDS + 1];
  const unsigned int n = a.offs[nreg];
  const unsigned int* offs = stage_offsets(a.offs, nreg, n, soffs);
  const long long nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long nfx = (nx + 1) * ny * nz, nfy = nx * (ny + 1) * nz;
  const double* Dd[3] = {a.D, a.D + NV * nfx, a.D + NV * (nfx + nfy)};
  double cfl_max = 0.0;
  bool cfl_bad = false;
  const unsigned int threads = gridDim.x * blockDim.x;
  for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += threads) {
    const int lo = find_segment(offs, nreg, i);
    const unsigned long long e = a.list[list_region_start(a, g, lo) + (i - offs[lo])];
    const long long c = (long long)(e >> 8);
    const unsigned cm = (unsigned)(e & 0xffu);
    const long long x = c % nx, y = (c / nx) % ny, z = c / (nx * ny);
    // the face below the cell along each direction (the one above is next)
    const long long lof[3] = {x + (nx + 1) * (y + ny * z), x + nx * (y + (ny + 1) * z), c};
    const long long step[3] = {1, nx, nx * ny};
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      if (!((cm >> f) & 1u)) continue;
      const int dir = f >> 1;
      const long long idx = lof[dir] + ((f & 1) ? step[dir] : 0);
      const double sg = (f & 1) ? -1.0 : 1.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += sg * Dd[dir][NV * idx + v];
    }
    double un[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      un[v] = a.out[v * g.ncell + c] + scale * (acc[v] * ph.inv_dx);
      a.out[v * g.ncell + c] = un[v];
    }
    if (OUT == OUT_RK && a.cfl != nullptr) {
      const double m[3] = {un[1], un[2], un[3]};
      cfl_max = nan_max(cfl_max, cfl_speed<3>(un[0], m, un[4], ph.gamma, cfl_bad));
    }
  }
  if (OUT == OUT_RK && a.cfl != nullptr) cfl_commit_wave(a.cfl, cfl_max, cfl_bad);
}

// Every face WENO, face-once form: the change of each face's flux (WENO
// minus linear) computed once, into D[v][face] with the faces of direction
// DIR numbered x + ex * (y + ey * z), (ex, ey, ez) the grid extents with one
// more face along DIR (face f lies between cells f-1 and f).  A face's change
// depends on its position only, so it equals what the per-cell kernel
// computes for either of its cells.
// W: the weighting of the reconstruction fixed at compile time (W_*), or -1
// to read it at run time.
template <int OUT, int DIR, int SPLIT, int HYB, int W>
__global__ __launch_bounds__(128) void weno_face3d_kernel(FusedArgs a, KGrid g, KPhys ph, double* D) {
  constexpr int NV = 5;
  if (OUT == OUT_RK && !(a.ctl->dt > 0.0)) return;
  const long long ex = g.n[0] + (DIR == 0), ey = g.n[1] + (DIR == 1), ez = g.n[2] + (DIR == 2);
  const long long nf = ex * ey * ez;
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += step) {
    const int x = (int)(i % ex);
    const int y = (int)((i / ex) % ey);
    const int z = (int)(i / (ex * ey));
    double dF[NV];
    face_delta<NV, DIR, SPLIT, HYB, W>(a.Uk, g, ph, a.ctl->lf_bits[DIR], x, y, z, 0, dF);
#pragma unroll
    for (int v = 0; v < NV; ++v) D[v * nf + i] = dF[v];
  }
}

// Face-once form, per cell: the six face changes from D summed in the fixed
// order x-, x+, y-, y+, z-, z+ (+ below, - above) and added to the output
// exactly as weno_fix3d_kernel adds them (the same bits); the CFL speed of
// the new state is folded for every cell; the next stage's list counter is
// cleared.
template <int OUT>
__global__ __launch_bounds__(256) void weno_sum3d_kernel(FusedArgs a, KGrid g, KPhys ph,
                                                         const double* Dx, const double* Dy,
                                                         const double* Dz) {
  constexpr int NV = 5;
  if (a.list_clear != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.list_clear = 0u;
  double scale = 1.0;
  if (OUT == OUT_RK) {
    const double dt = a.ctl->dt;
    if (!(dt > 0.0)) return;
    scale = a.rk_b * dt;
  }
  const long long nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long nfx = (nx + 1) * ny * nz, nfy = nx * (ny + 1) * nz, nfz = nx * ny * (nz + 1);
  double cfl_max = 0.0;
  bool cfl_bad = false;
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < g.ncell; c += step) {
    const long long x = c % nx, y = (c / nx) % ny, z = c / (nx * ny);
    const long long fx = x + (nx + 1) * (y + ny * z);
    const long long fy = x + nx * (y + (ny + 1) * z);
    const long long fz = c;
    const long long lo[3] = {fx, fy, fz}, hi[3] = {fx + 1, fy + nx, fz + nx * ny};
    const double* Dd[3] = {Dx, Dy, Dz};
    const long long nf[3] = {nfx, nfy, nfz};
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int dir = f >> 1;
      const long long idx = (f & 1) ? hi[dir] : lo[dir];
      const double sg = (f & 1) ? -1.0 : 1.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += sg * Dd[dir][v * nf[dir] + idx];
    }
    double un[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      un[v] = a.out[v * g.ncell + c] + scale * (acc[v] * ph.inv_dx);
      a.out[v * g.ncell + c] = un[v];
    }
    if (OUT == OUT_RK && a.cfl != nullptr) {
      const double m[3] = {un[1], un[2], un[3]};
      cfl_max = nan_max(cfl_max, cfl_speed<3>(un[0], m, un[4], ph.gamma, cfl_bad));
    }
  }
  if (OUT == OUT_RK && a.cfl != nullptr) cfl_commit_wave(a.cfl, cfl_max, cfl_bad);
}

// Exclusive prefix sums of the per-workgroup list counts: offs[r] = entries
// of the regions before r, offs[nreg] = all entries.  One workgroup of 1024
// threads, each summing a contiguous run of counts.
__device__ __forceinline__ void scan_counts(const unsigned int* counts, int nreg, unsigned int* offs,
                                            unsigned int* part) {
  const int t = threadIdx.x;
  const int per = (nreg + 1023) / 1024;
  const int b = t * per, e = min(b + per, nreg);
  unsigned int sum = 0u;
  for (int r = b; r < e; ++r) sum += counts[r];
  part[t] = sum;
  __syncthreads();
  // inclusive scan of the 1024 partial sums (Hillis-Steele)
  for (int d = 1; d < 1024; d <<= 1) {
    const unsigned int v = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned int run = t > 0 ? part[t - 1] : 0u;
  for (int r = b; r < e; ++r) {
    offs[r] = run;
    run += counts[r];
  }
  if (t == 1023) offs[nreg] = part[1023];
}

static __global__ __launch_bounds__(1024) void list_scan_kernel(const unsigned int* counts, int nreg,
                                                                unsigned int* offs) {
  __shared__ unsigned int part[1024];
  scan_counts(counts, nreg, offs, part);
}

// Both offset arrays of the face-list corrections (cells: counts -> offs;
// faces: counts_f -> offs_f over the 3 nreg (direction, region) segments) in
// one launch; nothing to do when the stage listed no cell.
static __global__ __launch_bounds__(1024) void list_scan2_kernel(FusedArgs a, int nreg) {
  __shared__ unsigned int part[1024];
  if (*a.list_n == 0u) return;
  scan_counts(a.counts, nreg, a.offs, part);
  __syncthreads();
  scan_counts(a.counts_f, 3 * nreg, a.offs_f, part);
}

[[maybe_unused]] static __global__ void reset_list_kernel(unsigned int* list_n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *list_n = 0u;
}

}  // namespace wl2
