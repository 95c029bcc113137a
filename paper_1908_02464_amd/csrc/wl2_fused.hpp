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
// light record.  The WENO branch of a flagged face is taken in place.
// Tiles are numbered so that the workgroups resident on one XCD (dispatch is
// round-robin over the 8 XCDs) take a contiguous range of tiles and share
// their halos in that XCD's L2.
#pragma once
#include "wl2_device.hpp"
#include "wl2_fused_launch.hpp"

namespace wl2 {

constexpr int FT_THREADS = 256;
constexpr int FT_OWN = FT_X * FT_Y;              // 240 column owners
constexpr int FP_X = FT_X + 6, FP_Y = FT_Y + 6;  // LDS plane pitch (with halo)
constexpr int FP_N = FP_X * FP_Y;
constexpr int NXF = (FT_X + 1) * FT_Y;           // 255 x faces per plane
constexpr int NYF = FT_X * (FT_Y + 1);           // 256 y faces per plane
constexpr int NHALO = 6 * FT_Y + 6 * FT_X;       // 186 halo cells per plane

// 1/x and 1/sqrt(x) from the hardware seeds refined by two Newton steps (the
// seed error squares each step; the result is within a few ulp, not
// correctly rounded).
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
  }
  return r;
}

__device__ __forceinline__ double fast_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
  }
  return y;
}

template <int NV>
struct LRec {
  double U[NV];
  double p, c, iw;  // pressure, sound speed, 1/sqrt(rho)
};

template <int NV>
__device__ __forceinline__ void make_lrec(const double (&u)[NV], const KPhys& ph, LRec<NV>& r) {
  constexpr int DIM = NV - 2;
  const double iw = fast_rsqrt(u[0]);
  const double ir = iw * iw;
  double m2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) m2 += u[1 + k] * u[1 + k];
  const double p = ph.gm1 * (u[NV - 1] - 0.5 * ir * m2);
  const double c2 = ph.gamma * p * ir;
  r.c = c2 * fast_rsqrt(c2);
  r.p = p;
  r.iw = iw;
#pragma unroll
  for (int v = 0; v < NV; ++v) r.U[v] = u[v];
}

// Flux along DIR and normal velocity from a light record.
template <int NV, int DIR>
__device__ __forceinline__ void lflux(const LRec<NV>& r, double (&F)[NV], double& un) {
  constexpr int DIM = NV - 2;
  un = r.U[1 + DIR] * (r.iw * r.iw);
  F[0] = r.U[1 + DIR];
#pragma unroll
  for (int k = 0; k < DIM; ++k) F[1 + k] = un * r.U[1 + k] + (k == DIR ? r.p : 0.0);
  F[NV - 1] = (r.U[NV - 1] + r.p) * un;
}

template <int NV, int DIR>
__device__ __forceinline__ void to_cellrec(const LRec<NV>& r, CellRec<NV>& c) {
#pragma unroll
  for (int v = 0; v < NV; ++v) c.U[v] = r.U[v];
  lflux<NV, DIR>(r, c.F, c.un);
  c.c = r.c;
  c.iw = r.iw;
  c.p = r.p;
}

template <int NV, int DIR>
__device__ __forceinline__ void roe_light(const LRec<NV>& L, const LRec<NV>& R, const KPhys& ph,
                                          Roe<NV>& s) {
  constexpr int DIM = NV - 2;
  const double wl = L.U[0] * L.iw, wr = R.U[0] * R.iw;
  const double is = fast_rcp(wl + wr);
  double q = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    s.u[k] = (L.U[1 + k] * L.iw + R.U[1 + k] * R.iw) * is;
    q += s.u[k] * s.u[k];
  }
  s.q = 0.5 * q;
  s.H = ((L.U[NV - 1] + L.p) * L.iw + (R.U[NV - 1] + R.p) * R.iw) * is;
  const double c2 = ph.gm1 * (s.H - s.q);
  s.ic = fast_rsqrt(c2);
  s.c = c2 * s.ic;
  s.b1 = ph.gm1 * s.ic * s.ic;
  s.b2 = s.b1 * s.q;
  s.irho = L.iw * R.iw;
}

// Linear-branch flux of one face from six light records; returns the mask
// of fields whose detector asks for the nonlinear flux.
// `src.get(m, rec)` supplies stencil cell m = 0..5 (j-2 .. j+3); cells are
// requested in the pairs (0,5), (1,4), (2,3) so only two are live at a time.
// SPLIT / HYB: compile-time splitting and switch modes, or -1 to read them
// from ph at run time.
template <int NV, int DIR, int SPLIT, int HYB, class Src>
__device__ __forceinline__ unsigned face_linear_l(const Src& src, const KPhys& ph, double eps_thr,
                                                  const unsigned long long* lfb, double (&Fh)[NV]) {
  const int split = SPLIT >= 0 ? SPLIT : ph.split;
  const int hybrid = HYB >= 0 ? HYB : ph.hybrid;
  double dU5[NV], Fc6[NV];
  double am, a0, ap;
  LRec<NV> c2, c3;
  {
    LRec<NV> c0, c5;
    src.get(0, c0);
    src.get(5, c5);
    double F0[NV], F5[NV], u0, u5;
    lflux<NV, DIR>(c0, F0, u0);
    lflux<NV, DIR>(c5, F5, u5);
    am = fmax(fabs(u0 - c0.c), fabs(u5 - c5.c));
    a0 = fmax(fabs(u0), fabs(u5));
    ap = fmax(fabs(u0 + c0.c), fabs(u5 + c5.c));
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      dU5[i] = c0.U[i] - c5.U[i];
      Fc6[i] = F0[i] + F5[i];
    }
  }
  {
    LRec<NV> c1, c4;
    src.get(1, c1);
    src.get(4, c4);
    double F1[NV], F4[NV], u1, u4;
    lflux<NV, DIR>(c1, F1, u1);
    lflux<NV, DIR>(c4, F4, u4);
    am = fmax(am, fmax(fabs(u1 - c1.c), fabs(u4 - c4.c)));
    a0 = fmax(a0, fmax(fabs(u1), fabs(u4)));
    ap = fmax(ap, fmax(fabs(u1 + c1.c), fabs(u4 + c4.c)));
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      dU5[i] += 5.0 * (c4.U[i] - c1.U[i]);
      Fc6[i] -= 8.0 * (F1[i] + F4[i]);
    }
  }
  src.get(2, c2);
  src.get(3, c3);
  {
    double F2[NV], F3[NV], u2, u3;
    lflux<NV, DIR>(c2, F2, u2);
    lflux<NV, DIR>(c3, F3, u3);
    am = fmax(am, fmax(fabs(u2 - c2.c), fabs(u3 - c3.c)));
    a0 = fmax(a0, fmax(fabs(u2), fabs(u3)));
    ap = fmax(ap, fmax(fabs(u2 + c2.c), fabs(u3 + c3.c)));
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      dU5[i] += 10.0 * (c2.U[i] - c3.U[i]);
      Fc6[i] = (Fc6[i] + 37.0 * (F2[i] + F3[i])) * (1.0 / 60.0);
    }
  }
  Roe<NV> s;
  roe_light<NV, DIR>(c2, c3, ph, s);
  double a[NV];
  if (split == SPLIT_LLF) {
    a[0] = am;
#pragma unroll
    for (int k = 1; k < NV - 1; ++k) a[k] = a0;
    a[NV - 1] = ap;
  } else if (split == SPLIT_ROE) {
    a[0] = fabs(s.u[DIR] - s.c);
#pragma unroll
    for (int k = 1; k < NV - 1; ++k) a[k] = fabs(s.u[DIR]);
    a[NV - 1] = fabs(s.u[DIR] + s.c);
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] = __longlong_as_double((long long)lfb[k]);
  }
  double dv[NV], d[NV];
  project<NV, DIR>(s, dU5, dv);
  unsigned weno = 0;
  double smax = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    dv[k] *= (1.0 / 60.0);
    const double t = dv[k] * s.irho;
    const double sig = t * t;  // Eq.(30)
    smax = fmax(smax, sig);
    if (!(sig < eps_thr)) weno |= 1u << k;
    d[k] = a[k] * dv[k];
  }
  if (hybrid == HYB_PER_FACE) weno = (smax < eps_thr) ? 0u : ((1u << NV) - 1u);
  else if (hybrid == HYB_WENO_ONLY) weno = (1u << NV) - 1u;
  else if (hybrid == HYB_LINEAR_ONLY) weno = 0u;
  double Rd[NV];
  back_project<NV, DIR>(s, d, Rd);
#pragma unroll
  for (int i = 0; i < NV; ++i) Fh[i] = Fc6[i] + Rd[i];
  return weno;
}

struct V5 {
  double v[5];
};

struct FusedArgs {
  const double* Uk;   // stage input
  double* out;        // RK: U^(k+1); RHS: dU/dt
  const double* Un;   // RK: U^n (read when rk_a != 0)
  const StepCtl* ctl;
  double rk_a, rk_b;
  int zc;             // planes per workgroup
  int tiles_x, tiles_y;
  unsigned long long* list;  // cells next to a face that needs the WENO flux
  unsigned int* list_n;      // number of entries in list
  StepCtl* cfl;              // RK: if set, fold the CFL speed of the new state
                             // into cfl->smax_bits / status (next step's dt)
};

// Index of a line position clamped to [-3, n+2] and mapped through the
// boundary rule; flip set for mirror ghosts.
__device__ __forceinline__ int ghost_clamped(int k, int n, int lo, int hi, bool& flip) {
  k = k < -3 ? -3 : (k > n + 2 ? n + 2 : k);
  return ghost_index(k, n, lo, hi, flip);
}

template <int NV>
__device__ __forceinline__ void lds_put(double (*srec)[FP_N], int idx, const LRec<NV>& r) {
#pragma unroll
  for (int v = 0; v < NV; ++v) srec[v][idx] = r.U[v];
  srec[NV][idx] = r.p;
  srec[NV + 1][idx] = r.c;
  srec[NV + 2][idx] = r.iw;
}

template <int NV>
__device__ __forceinline__ void lds_get(double (*srec)[FP_N], int idx, LRec<NV>& r) {
#pragma unroll
  for (int v = 0; v < NV; ++v) r.U[v] = srec[v][idx];
  r.p = srec[NV][idx];
  r.c = srec[NV + 1][idx];
  r.iw = srec[NV + 2][idx];
}

// Stencil accessors for face_linear_l.
template <int NV>
struct WinSrc {  // the owner's z window (registers)
  const LRec<NV>&w0, &w1, &w2, &w3, &w4, &w5;
  __device__ __forceinline__ void get(int m, LRec<NV>& r) const {
    r = m == 0 ? w0 : m == 1 ? w1 : m == 2 ? w2 : m == 3 ? w3 : m == 4 ? w4 : w5;
  }
};

template <int NV>
struct LdsSrc {  // six cells of the LDS plane at base + m*stride
  double (*srec)[FP_N];
  int base, stride;
  __device__ __forceinline__ void get(int m, LRec<NV>& r) const {
    lds_get<NV>(srec, base + m * stride, r);
  }
};

// Nonlinear (WENO-L2IS) correction of one flagged face, field by field:
// for each field k in `mask`, the left eigenvector row L^k is formed, the six
// stencil cells are projected (Eq.(20)), split (Eq.(21)) and reconstructed
// (Eq.(22)-(23)); the change with respect to the linear flux of that field is
// back-projected (Eq.(24)).  Only one row and twelve split values are live.
template <int NV, int DIR, int K, class Src>
__device__ __forceinline__ double lean_field(const Src& src, const Roe<NV>& s, double al, double dvk,
                                             double LFk, const KPhys& ph) {
  double r[NV];
  left_row<NV, DIR, K>(s, r);
  double fp[6], fm[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    LRec<NV> cm;
    src.get(m, cm);
    double F[NV], un;
    lflux<NV, DIR>(cm, F, un);
    const double vv = dot<NV>(r, cm.U);
    const double gg = dot<NV>(r, F);
    fp[m] = 0.5 * (gg + al * vv);
    fm[m] = 0.5 * (gg - al * vv);
  }
  const double t = dvk * s.irho;
  const double lam = ph.c_reg * (t * t);  // Eq.(32)
  const double fw = weno_l2is(fp[0], fp[1], fp[2], fp[3], fp[4], lam, ph.eps_w) +
                    weno_l2is(fm[5], fm[4], fm[3], fm[2], fm[1], lam, ph.eps_w);
  return fw - (LFk + al * dvk);
}

template <int NV, int DIR, class Src>
__device__ __forceinline__ void lean_correction(const Src& src, unsigned mask, const KPhys& ph,
                                                const unsigned long long* lfb, double (&dF)[NV]) {
  double dU5[NV], Fc6[NV];
  double am = 0.0, a0 = 0.0, ap = 0.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) dU5[i] = Fc6[i] = 0.0;
  constexpr double cu[6] = {1.0, -5.0, 10.0, -10.0, 5.0, -1.0};
  constexpr double cf[6] = {1.0, -8.0, 37.0, 37.0, -8.0, 1.0};
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    LRec<NV> cm;
    src.get(m, cm);
    double F[NV], un;
    lflux<NV, DIR>(cm, F, un);
    am = fmax(am, fabs(un - cm.c));
    a0 = fmax(a0, fabs(un));
    ap = fmax(ap, fabs(un + cm.c));
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      dU5[i] += cu[m] * cm.U[i];
      Fc6[i] += cf[m] * F[i];
    }
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) Fc6[i] *= (1.0 / 60.0);
  Roe<NV> s;
  {
    LRec<NV> c2, c3;
    src.get(2, c2);
    src.get(3, c3);
    roe_light<NV, DIR>(c2, c3, ph, s);
  }
  double a[NV];
  if (ph.split == SPLIT_LLF) {
    a[0] = am;
#pragma unroll
    for (int k = 1; k < NV - 1; ++k) a[k] = a0;
    a[NV - 1] = ap;
  } else if (ph.split == SPLIT_ROE) {
    a[0] = fabs(s.u[DIR] - s.c);
#pragma unroll
    for (int k = 1; k < NV - 1; ++k) a[k] = fabs(s.u[DIR]);
    a[NV - 1] = fabs(s.u[DIR] + s.c);
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] = __longlong_as_double((long long)lfb[k]);
  }
  double dv[NV], LF[NV], del[NV];
  project<NV, DIR>(s, dU5, dv);
  project<NV, DIR>(s, Fc6, LF);
#define WL2_LF(K)                                                                          \
  del[K] = ((mask >> K) & 1u)                                                              \
               ? lean_field<NV, DIR, K>(src, s, a[K], dv[K] * (1.0 / 60.0), LF[K], ph)    \
               : 0.0;
  WL2_LF(0) WL2_LF(1) WL2_LF(2) WL2_LF(3) WL2_LF(4)
#undef WL2_LF
  back_project<NV, DIR>(s, del, dF);
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
  double (*swin)[NV + 3][FT_OWN];
  int slot0, slot1, col;
  const LRec<NV>&r0, &r1, &r2, &r3;
  __device__ __forceinline__ void ring(int slot, LRec<NV>& r) const {
#pragma unroll
    for (int v = 0; v < NV; ++v) r.U[v] = swin[slot][v][col];
    r.p = swin[slot][NV][col];
    r.c = swin[slot][NV + 1][col];
    r.iw = swin[slot][NV + 2][col];
  }
  __device__ __forceinline__ void get(int m, LRec<NV>& r) const {
    if (m == 0) ring(slot0, r);
    else if (m == 1) ring(slot1, r);
    else r = m == 2 ? r0 : m == 3 ? r1 : m == 4 ? r2 : r3;
  }
};

// WPE: target waves per SIMD.  SPLIT / HYB: compile-time modes (-1: runtime).
template <int OUT, int WPE, int SPLIT, int HYB>
__global__ __launch_bounds__(FT_THREADS, WPE) void fused3d_kernel(FusedArgs a, KGrid g, KPhys ph) {
  constexpr int NV = 5;
  __shared__ double srec[NV + 3][FP_N];      // plane z with halo
  __shared__ double sfx[NV][NXF];            // x-face fluxes of plane z
  __shared__ double sfy[NV][NYF];            // y-face fluxes of plane z
  __shared__ double swin[2][NV + 3][FT_OWN]; // two oldest cells of each z window
  __shared__ unsigned char sgx[NXF], sgy[NYF];  // face needs the nonlinear flux

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
  const int lds_own = (oy + 3) * FP_X + (ox + 3);
  const Col ocol = make_col(g, gx, gy);
  const long long oout = (long long)gx + (long long)gy * g.stride[1];

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
  const int lds_halo = (hr + 3) * FP_X + (hc + 3);
  const Col hcol = make_col(g, x0 + hc, y0 + hr);

  // owner registers: r0..r3 = cells z-1 .. z+2 at the top of iteration z;
  // the ring holds cell c in slot (c & 1)
  LRec<NV> r0, r1, r2, r3;
  double Fzp[NV];
  bool zprev = false;  // face z - 1/2 needs the nonlinear flux
  double upre[NV], hpre[NV];
  double cfl_max = 0.0;  // CFL speed of the cells written here (a.cfl set)
  bool cfl_bad = false;
  double unp[NV] = {};  // U^n of cell z (RK stages 2, 3), loaded a phase ahead
  if (owner) {
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
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      swin[s3][v][t] = c0.U[v];
      swin[s2][v][t] = c1.U[v];
    }
    swin[s3][NV][t] = c0.p;
    swin[s3][NV + 1][t] = c0.c;
    swin[s3][NV + 2][t] = c0.iw;
    swin[s2][NV][t] = c1.p;
    swin[s2][NV + 1][t] = c1.c;
    swin[s2][NV + 2][t] = c1.iw;
    // face z0 - 1/2 (cells z0-3 .. z0+2): window c0, c1, r0, r1, r2, r3
    const WinSrc<NV> src{c0, c1, r0, r1, r2, r3};
    zprev = face_linear_l<NV, 2, SPLIT, HYB>(src, ph, ph.eps_thr[2], lfz, Fzp) != 0u;
    load_col_raw<NV>(a.Uk, g, ocol, z0 + 3, upre);
  }
  if (t < NHALO) load_col_raw<NV>(a.Uk, g, hcol, z0, hpre);

  for (int z = z0; z < z1; ++z) {
    if (owner) {
      // retire cell z-1 into the ring (overwrites cell z-3), then shift:
      // registers become cells z .. z+3
      const int sl = (z - 1) & 1;
#pragma unroll
      for (int v = 0; v < NV; ++v) swin[sl][v][t] = r0.U[v];
      swin[sl][NV][t] = r0.p;
      swin[sl][NV + 1][t] = r0.c;
      swin[sl][NV + 2][t] = r0.iw;
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
    if (t < NHALO) {
      LRec<NV> hrec;
      col_flip<NV>(g, hcol, z, hpre);
      make_lrec<NV>(hpre, ph, hrec);
      lds_put<NV>(srec, lds_halo, hrec);
      asm volatile("" ::: "memory");  // as above: the prefetch after the last use
      load_col_raw<NV>(a.Uk, g, hcol, z + 1, hpre);
    }
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    // x faces: thread t < 255 -> row t/17, face fx = t%17 at x0 + fx - 1/2
    if (t < NXF) {
      const int row = t / (FT_X + 1), fx = t % (FT_X + 1);
      const int base = (row + 3) * FP_X + fx;
      const LdsSrc<NV> src{srec, base, 1};
      double F[NV];
      sgx[t] = face_linear_l<NV, 0, SPLIT, HYB>(src, ph, ph.eps_thr[0], lfx, F) != 0u;
#pragma unroll
      for (int v = 0; v < NV; ++v) sfx[v][t] = F[v];
    }
    __builtin_amdgcn_sched_barrier(0);
    // y faces: thread t -> column t%16, face fy = t/16 at y0 + fy - 1/2
    {
      const int col = t % FT_X, fy = t / FT_X;
      const int base = fy * FP_X + col + 3;
      const LdsSrc<NV> src{srec, base, FP_X};
      double F[NV];
      sgy[t] = face_linear_l<NV, 1, SPLIT, HYB>(src, ph, ph.eps_thr[1], lfy, F) != 0u;
#pragma unroll
      for (int v = 0; v < NV; ++v) sfy[v][t] = F[v];
    }
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    if (owner) {
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
      // wave-aggregated append to the correction list
      const unsigned long long ball = __ballot(cm != 0u);
      if (ball) {
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((long long)ball) - 1;
        unsigned int basei = 0;
        if (lane == leader) basei = atomicAdd(a.list_n, (unsigned int)__popcll(ball));
        basei = __shfl(basei, leader, 64);
        if (cm) {
          const unsigned int rank = __popcll(ball & ((1ull << lane) - 1ull));
          a.list[basei + rank] = ((unsigned long long)off << 8) | cm;
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
    }
  }
  if (OUT == OUT_RK && a.cfl != nullptr) cfl_commit_wave(a.cfl, cfl_max, cfl_bad);
}

// Nonlinear correction of one face of cell (x, y, z) along DIR: side 0 is
// the face below the cell, side 1 the face above.  Returns the change of the
// face flux (WENO minus linear, Eq.(33) per field).
template <int NV, int DIR, int SPLIT, int HYB>
__device__ __forceinline__ void face_delta(const double* U, const KGrid& g, const KPhys& ph,
                                           const unsigned long long* lfb, int x, int y, int z,
                                           int side, double (&dF)[NV]) {
  struct Src {
    const double* U;
    const KGrid* g;
    const KPhys* ph;
    int c[3];
    __device__ __forceinline__ void get(int m, LRec<NV>& r) const {
      double u[NV];
      bool flip;
      const int k = ghost_clamped(c[DIR] + m, g->n[DIR], g->bc_lo[DIR], g->bc_hi[DIR], flip);
      int p[3] = {c[0], c[1], c[2]};
      p[DIR] = k;
      const long long off = p[0] + (long long)p[1] * g->stride[1] + (long long)p[2] * g->stride[2];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = U[v * g->ncell + off];
      if (flip) u[1 + DIR] = -u[1 + DIR];
      make_lrec<NV>(u, *ph, r);
    }
  } src{U, &g, &ph, {x, y, z}};
  // face below the cell: stencil starts 3 cells below; face above: 2 below
  src.c[DIR] += side ? -2 : -3;
  double Flin[NV];
  const unsigned mask =
      face_linear_l<NV, DIR, SPLIT, HYB>(src, ph, ph.eps_thr[DIR], lfb, Flin);
  if (mask) {
    lean_correction<NV, DIR>(src, mask, ph, lfb, dF);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) dF[v] = 0.0;
  }
}

// One thread per listed cell: add the nonlinear part of the flux of its
// flagged faces, in the fixed order x-, x+, y-, y+, z-, z+, to the output
// (scaled by rk_b dt for a stage, 1 for dU/dt).  Each cell is owned by one
// thread, so the result does not depend on scheduling.
template <int OUT, int SPLIT, int HYB>
__global__ __launch_bounds__(128) void weno_fix3d_kernel(FusedArgs a, KGrid g, KPhys ph) {
  constexpr int NV = 5;
  double scale = 1.0;
  if (OUT == OUT_RK) {
    const double dt = a.ctl->dt;
    if (!(dt > 0.0)) return;
    scale = a.rk_b * dt;
  }
  const unsigned int n = *a.list_n;
  double cfl_max = 0.0;
  bool cfl_bad = false;
  for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const unsigned long long e = a.list[i];
    const long long off = (long long)(e >> 8);
    const unsigned cm = (unsigned)(e & 0xffu);
    const int x = (int)(off % g.n[0]);
    const int y = (int)((off / g.n[0]) % g.n[1]);
    const int z = (int)(off / g.stride[2]);
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int f = 0; f < 6; ++f) {
      if (!((cm >> f) & 1u)) continue;
      const int dir = f >> 1, side = f & 1;
      double dF[NV];
      if (dir == 0) face_delta<NV, 0, SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[0], x, y, z, side, dF);
      else if (dir == 1) face_delta<NV, 1, SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[1], x, y, z, side, dF);
      else face_delta<NV, 2, SPLIT, HYB>(a.Uk, g, ph, a.ctl->lf_bits[2], x, y, z, side, dF);
      // dU = -(F_{+} - F_{-}) / dx: the face below adds, the face above subtracts
      const double sg = side ? -1.0 : 1.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += sg * dF[v];
    }
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
  if (OUT == OUT_RK && a.cfl != nullptr) cfl_commit_wave(a.cfl, cfl_max, cfl_bad);
}

[[maybe_unused]] static __global__ void reset_list_kernel(unsigned int* list_n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *list_n = 0u;
}

}  // namespace wl2
