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

namespace wl2 {

constexpr int FT_X = 16, FT_Y = 15, FT_THREADS = 256;
constexpr int FT_OWN = FT_X * FT_Y;              // 240 column owners
constexpr int FP_X = FT_X + 6, FP_Y = FT_Y + 6;  // LDS plane pitch (with halo)
constexpr int FP_N = FP_X * FP_Y;
constexpr int NXF = (FT_X + 1) * FT_Y;           // 255 x faces per plane
constexpr int NYF = FT_X * (FT_Y + 1);           // 256 y faces per plane
constexpr int NHALO = 6 * FT_Y + 6 * FT_X;       // 186 halo cells per plane

// 1/x and 1/sqrt(x) from the hardware seeds refined by Newton steps (not
// correctly rounded; a few ulp, see DESIGN notes on precision).
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
  }
  return r;
}

__device__ __forceinline__ double fast_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
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
template <int NV, int DIR, class Src>
__device__ __forceinline__ unsigned face_linear_l(const Src& src, const KPhys& ph, double eps_thr,
                                                  const unsigned long long* lfb, double (&Fh)[NV]) {
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
  if (ph.hybrid == HYB_PER_FACE) weno = (smax < eps_thr) ? 0u : ((1u << NV) - 1u);
  else if (ph.hybrid == HYB_WENO_ONLY) weno = (1u << NV) - 1u;
  else if (ph.hybrid == HYB_LINEAR_ONLY) weno = 0u;
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
  int tiles_x, tiles_y, nzc;
};

// Index of a line position clamped to [-3, n+2] and mapped through the
// boundary rule; flip set for mirror ghosts.
__device__ __forceinline__ int ghost_clamped(int k, int n, int lo, int hi, bool& flip) {
  k = k < -3 ? -3 : (k > n + 2 ? n + 2 : k);
  return ghost_index(k, n, lo, hi, flip);
}

template <int NV>
__device__ __forceinline__ void load_xyz(const double* __restrict__ U, const KGrid& g, int x, int y,
                                         int z, double (&u)[NV]) {
  bool fx, fy, fz;
  const int ix = ghost_clamped(x, g.n[0], g.bc_lo[0], g.bc_hi[0], fx);
  const int iy = ghost_clamped(y, g.n[1], g.bc_lo[1], g.bc_hi[1], fy);
  const int iz = ghost_clamped(z, g.n[2], g.bc_lo[2], g.bc_hi[2], fz);
  const long long off = ix + (long long)iy * g.stride[1] + (long long)iz * g.stride[2];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = U[v * g.ncell + off];
  if (fx) u[1] = -u[1];
  if (fy) u[2] = -u[2];
  if (fz) u[3] = -u[3];
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

// WPE: target waves per SIMD (1: no register spills; 2: twice the
// resident waves with some spilling).  Picked per context by tuning.
template <int OUT, int WPE>
__global__ __launch_bounds__(FT_THREADS, WPE) void fused3d_kernel(FusedArgs a, KGrid g, KPhys ph) {
  constexpr int NV = 5;
  __shared__ double srec[NV + 3][FP_N];
  __shared__ double sfx[NV][NXF];
  __shared__ double sfy[NV][NYF];

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

  // z window of the owner's column: cells z-2 .. z+3 after each push
  LRec<NV> w0, w1, w2, w3, w4, w5;
  double Fzp[NV];
  double upre[NV], hpre[NV];
  if (owner) {
    double u[NV];
    load_xyz<NV>(a.Uk, g, gx, gy, z0 - 3, u);
    make_lrec<NV>(u, ph, w0);
    load_xyz<NV>(a.Uk, g, gx, gy, z0 - 2, u);
    make_lrec<NV>(u, ph, w1);
    load_xyz<NV>(a.Uk, g, gx, gy, z0 - 1, u);
    make_lrec<NV>(u, ph, w2);
    load_xyz<NV>(a.Uk, g, gx, gy, z0, u);
    make_lrec<NV>(u, ph, w3);
    load_xyz<NV>(a.Uk, g, gx, gy, z0 + 1, u);
    make_lrec<NV>(u, ph, w4);
    load_xyz<NV>(a.Uk, g, gx, gy, z0 + 2, u);
    make_lrec<NV>(u, ph, w5);
    // face z0 - 1/2 (cells z0-3 .. z0+2)
    const WinSrc<NV> src{w0, w1, w2, w3, w4, w5};
    const unsigned m = face_linear_l<NV, 2>(src, ph, ph.eps_thr[2], lfz, Fzp);
    if (m) {
      double dF[NV];
      lean_correction<NV, 2>(src, m, ph, lfz, dF);
#pragma unroll
      for (int v = 0; v < NV; ++v) Fzp[v] += dF[v];
    }
    load_xyz<NV>(a.Uk, g, gx, gy, z0 + 3, upre);
  }
  if (t < NHALO) load_xyz<NV>(a.Uk, g, x0 + hc, y0 + hr, z0, hpre);

  for (int z = z0; z < z1; ++z) {
    if (owner) {
      // push cell z+3; window becomes z-2 .. z+3
      w0 = w1;
      w1 = w2;
      w2 = w3;
      w3 = w4;
      w4 = w5;
      make_lrec<NV>(upre, ph, w5);
      if (z + 1 < z1) load_xyz<NV>(a.Uk, g, gx, gy, z + 4, upre);
      lds_put<NV>(srec, lds_own, w2);  // cell z
    }
    if (t < NHALO) {
      LRec<NV> hr_;
      make_lrec<NV>(hpre, ph, hr_);
      lds_put<NV>(srec, lds_halo, hr_);
      if (z + 1 < z1) load_xyz<NV>(a.Uk, g, x0 + hc, y0 + hr, z + 1, hpre);
    }
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    // x faces: thread t < 255 -> row t/17, face fx = t%17 at x0 + fx - 1/2
    if (t < NXF) {
      const int row = t / (FT_X + 1), fx = t % (FT_X + 1);
      const int base = (row + 3) * FP_X + fx;
      const LdsSrc<NV> src{srec, base, 1};
      double F[NV];
      const unsigned m = face_linear_l<NV, 0>(src, ph, ph.eps_thr[0], lfx, F);
      if (m) {
        double dF[NV];
        lean_correction<NV, 0>(src, m, ph, lfx, dF);
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] += dF[v];
      }
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
      const unsigned m = face_linear_l<NV, 1>(src, ph, ph.eps_thr[1], lfy, F);
      if (m) {
        double dF[NV];
        lean_correction<NV, 1>(src, m, ph, lfy, dF);
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] += dF[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) sfy[v][t] = F[v];
    }
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    double Fz[NV];
    if (owner) {
      // z face z + 1/2 from the register window
      const WinSrc<NV> src{w0, w1, w2, w3, w4, w5};
      const unsigned m = face_linear_l<NV, 2>(src, ph, ph.eps_thr[2], lfz, Fz);
      if (m) {
        double dF[NV];
        lean_correction<NV, 2>(src, m, ph, lfz, dF);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fz[v] += dF[v];
      }
    }
    if (valid) {
      const long long off = gx + (long long)gy * g.stride[1] + (long long)z * g.stride[2];
      const int ix = oy * (FT_X + 1) + ox;
      const int iy = oy * FT_X + ox;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double dU = ((sfx[v][ix] - sfx[v][ix + 1]) + (sfy[v][iy] - sfy[v][iy + FT_X]) +
                           (Fzp[v] - Fz[v])) * ph.inv_dx;
        if (OUT == OUT_RK) {
          double r = a.rk_b * (w2.U[v] + dt * dU);
          if (a.rk_a != 0.0) r += a.rk_a * a.Un[v * g.ncell + off];
          a.out[v * g.ncell + off] = r;
        } else {
          a.out[v * g.ncell + off] = dU;
        }
      }
    }
    if (owner) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Fzp[v] = Fz[v];
    }
  }
}

}  // namespace wl2
