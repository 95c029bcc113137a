// Face fluxes from "light" cell records (U, p, c, 1/sqrt(rho)): the linear
// branch of one face, its nonlinear (WENO-L2IS) correction, and the helpers
// they share.  Used by the fused 3D stage kernel and the 1D/2D row kernels;
// stencil cells come through small accessor objects (`src.get(m, rec)`), so
// the same arithmetic serves registers, LDS and global memory.
#pragma once
#include "wl2_device.hpp"

namespace wl2 {

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

// Intermediate quantities of a linear face that its nonlinear correction
// reuses: the Roe state, the splitting speeds, dv = L dU5 / 60 and Fc6.
template <int NV>
struct FaceState {
  Roe<NV> s;
  double a[NV], dv[NV], Fc6[NV];
};

// Linear-branch flux of one face from six light records, with its state for
// a correction; returns the mask of fields whose detector asks for the
// nonlinear flux.  Cells are requested in the pairs (0,5), (1,4), (2,3) so
// only two are live at a time.
template <int NV, int DIR, int SPLIT, int HYB, class Src>
__device__ __forceinline__ unsigned face_linear_st(const Src& src, const KPhys& ph, double eps_thr,
                                                   const unsigned long long* lfb, double (&Fh)[NV],
                                                   FaceState<NV>& st) {
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
      Fc6[i] += 37.0 * (F2[i] + F3[i]);  // 60 Fc6: the 1/60 is applied below
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
  // dv = L dU5 / 60 and Fc6 enter scaled by 60; the 1/60 is folded into
  // the detector scale, the splitting speeds and the final flux
  constexpr double k60 = 1.0 / 60.0;
  double dv[NV], d[NV], a60[NV];
  project<NV, DIR>(s, dU5, dv);
  const double irho60 = s.irho * k60;
  if (split == SPLIT_LLF) {
    const double am60 = a[0] * k60, a060 = a[1] * k60, ap60 = a[NV - 1] * k60;
    a60[0] = am60;
#pragma unroll
    for (int k = 1; k < NV - 1; ++k) a60[k] = a060;
    a60[NV - 1] = ap60;
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) a60[k] = a[k] * k60;
  }
  unsigned weno = 0;
  double smax = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double t = dv[k] * irho60;
    const double sig = t * t;  // Eq.(30)
    smax = fmax(smax, sig);
    if (!(sig < eps_thr)) weno |= 1u << k;
    d[k] = a60[k] * dv[k];
  }
  if (hybrid == HYB_PER_FACE) weno = (smax < eps_thr) ? 0u : ((1u << NV) - 1u);
  else if (hybrid == HYB_WENO_ONLY) weno = (1u << NV) - 1u;
  else if (hybrid == HYB_LINEAR_ONLY) weno = 0u;
  double Rd[NV];
  back_project<NV, DIR>(s, d, Rd);
#pragma unroll
  for (int i = 0; i < NV; ++i) Fh[i] = Fc6[i] * k60 + Rd[i];
  // the state in the paper's units for a nonlinear correction (dead code,
  // removed by the compiler, where the caller drops it)
  st.s = s;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    st.a[k] = a[k];
    st.dv[k] = dv[k] * k60;
    st.Fc6[k] = Fc6[k] * k60;
  }
  return weno;
}

// Linear-branch flux of one face from six light records; returns the mask
// of fields whose detector asks for the nonlinear flux.  `src.get(m, rec)`
// supplies stencil cell m = 0..5 (j-2 .. j+3).  SPLIT / HYB: compile-time
// splitting and switch modes, or -1 to read them from ph at run time.
template <int NV, int DIR, int SPLIT, int HYB, class Src>
__device__ __forceinline__ unsigned face_linear_l(const Src& src, const KPhys& ph, double eps_thr,
                                                  const unsigned long long* lfb, double (&Fh)[NV]) {
  FaceState<NV> st;
  return face_linear_st<NV, DIR, SPLIT, HYB>(src, ph, eps_thr, lfb, Fh, st);
}

// Index of a line position clamped to [-3, n+2] and mapped through the
// boundary rule; flip set for mirror ghosts.
__device__ __forceinline__ int ghost_clamped(int k, int n, int lo, int hi, bool& flip) {
  k = k < -3 ? -3 : (k > n + 2 ? n + 2 : k);
  return ghost_index(k, n, lo, hi, flip);
}

// Stencil accessor over six records held in registers.
template <int NV>
struct WinSrc {  // the owner's z window (registers)
  const LRec<NV>&w0, &w1, &w2, &w3, &w4, &w5;
  __device__ __forceinline__ void get(int m, LRec<NV>& r) const {
    r = m == 0 ? w0 : m == 1 ? w1 : m == 2 ? w2 : m == 3 ? w3 : m == 4 ? w4 : w5;
  }
};

// WENO-L2IS reconstruction at x_{j+1/2} from f_{j-2..j+2} (Eq.(5), (6),
// (11), (27), (28); optimal weights d = (0.4, 0.2, 0.3, 0.1)), the quotients
// through fast_rcp: the same formula as weno_l2is, a few ulp apart, with
// shorter dependency chains than correctly rounded division.  Every
// denominator is at least eps_w > 0 (the weight sum at least 1).  wts
// selects the comparison weights of Eq.(8) or Eq.(14)-(15) (lam unused).
__device__ __forceinline__ double weno_l2is_lr(double fm2, double fm1, double f0, double fp1,
                                               double fp2, double lam, double eps_w, int wts) {
  const double q0 = 0.5 * (f0 + fp1);
  const double q1 = 0.5 * (3.0 * f0 - fm1);
  const double q2 = (2.0 * f0 + 5.0 * fp1 - fp2) * (1.0 / 6.0);
  const double q3 = (2.0 * fm2 - 7.0 * fm1 + 11.0 * f0) * (1.0 / 6.0);
  const double d0 = fp1 - f0, d1 = f0 - fm1;
  const double b0 = d0 * d0, b1 = d1 * d1;
  const double s2a = f0 - 2.0 * fp1 + fp2, s2b = 3.0 * f0 - 4.0 * fp1 + fp2;
  const double s3a = fm2 - 2.0 * fm1 + f0, s3b = fm2 - 4.0 * fm1 + 3.0 * f0;
  const double b2 = (13.0 / 12.0) * s2a * s2a + 0.25 * s2b * s2b;
  const double b3 = (13.0 / 12.0) * s3a * s3a + 0.25 * s3b * s3b;
  const double t1 = (fp2 + fm2) - 4.0 * (fp1 + fm1) + 6.0 * f0;
  const double t2 = (fp2 - fm2) - 2.0 * (fp1 - fm1);
  const double tau5 = (13.0 / 12.0) * t1 * t1 + 0.25 * t2 * t2;
  const double e = fm1 - 2.0 * f0 + fp1;
  // one formula for the three weightings, the differences as selected
  // factors (no branch: both would hold their values in registers):
  // Eq.(28) d_k (1 + lam tau5 / (lam beta_k + E_k + eps)); Eq.(8) with lam
  // = 1 and E_k = 0; Eq.(14) with the numerator of the two-point stencils
  // multiplied by tau5 / (beta_01 + eps) of Eq.(15)
  const bool l2 = wts == W_L2IS;
  const double lv = l2 ? lam : 1.0;
  const double E01 = l2 ? e * e * (1.0 / 45.0) : 0.0;
  const double lt = lv * tau5;
  double n01 = lt;
  if (wts == W_IS_B01) {
    const double g = fm1 - fp1;
    n01 = tau5 * (tau5 * fast_rcp((13.0 / 12.0) * e * e + 0.25 * g * g + eps_w));
  }
  const double a0 = 0.4 * (1.0 + n01 * fast_rcp(lv * b0 + E01 + eps_w));
  const double a1 = 0.2 * (1.0 + n01 * fast_rcp(lv * b1 + E01 + eps_w));
  const double a2 = 0.3 * (1.0 + lt * fast_rcp(lv * b2 + eps_w));
  const double a3 = 0.1 * (1.0 + lt * fast_rcp(lv * b3 + eps_w));
  return (a0 * q0 + a1 * q1 + a2 * q2 + a3 * q3) * fast_rcp((a0 + a1) + (a2 + a3));
}

// Nonlinear (WENO-L2IS) correction of one flagged face, field by field:
// for each field k in `mask`, the left eigenvector row L^k is formed, the six
// stencil cells are projected (Eq.(20)), split (Eq.(21)) and reconstructed
// (Eq.(22)-(23)); the change with respect to the linear flux of that field is
// back-projected (Eq.(24)).  Only one row and twelve split values are live.
// W: the weighting (W_*) fixed at compile time, or -1 to read ph.weights.
template <int NV, int DIR, int W, class Src>
__device__ __forceinline__ double lean_field_row(const Src& src, const double (&r)[NV], const Roe<NV>& s,
                                                 double al, double dvk, double LFk, const KPhys& ph) {
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
  const int wts = W >= 0 ? W : ph.weights;
  const double fw = weno_l2is_lr(fp[0], fp[1], fp[2], fp[3], fp[4], lam, ph.eps_w, wts) +
                    weno_l2is_lr(fm[5], fm[4], fm[3], fm[2], fm[1], lam, ph.eps_w, wts);
  return fw - (LFk + al * dvk);
}

template <int NV, int DIR, int K, int W, class Src>
__device__ __forceinline__ double lean_field(const Src& src, const Roe<NV>& s, double al, double dvk,
                                             double LFk, const KPhys& ph) {
  double r[NV];
  left_row<NV, DIR, K>(s, r);
  return lean_field_row<NV, DIR, W>(src, r, s, al, dvk, LFk, ph);
}

// Row k of L for a field k known only at run time: each candidate row with
// the expressions of left_row<NV, DIR, k>, then selected (the same bits, no
// branch for lanes that take different fields).
template <int NV, int DIR>
__device__ __forceinline__ void left_row_rt(const Roe<NV>& s, int k, double (&r)[NV]) {
  constexpr int DIM = NV - 2;
  const double sg = k == 0 ? 1.0 : -1.0;
  double ac[NV], en[NV], sh[NV];
  ac[0] = 0.5 * (s.b2 + sg * s.u[DIR] * s.ic);
#pragma unroll
  for (int j = 0; j < DIM; ++j) ac[1 + j] = 0.5 * (-s.b1 * s.u[j] - (j == DIR ? sg * s.ic : 0.0));
  ac[NV - 1] = 0.5 * s.b1;
  en[0] = 1.0 - s.b2;
#pragma unroll
  for (int j = 0; j < DIM; ++j) en[1 + j] = s.b1 * s.u[j];
  en[NV - 1] = -s.b1;
  const int comp = (k - 2 < DIR) ? k - 2 : k - 1;  // shear field k-2: its momentum component
  double uc = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) uc = j == comp ? s.u[j] : uc;
  sh[0] = -uc * s.ic;
#pragma unroll
  for (int j = 0; j < DIM; ++j) sh[1 + j] = (j == comp) ? s.ic : 0.0;
  sh[NV - 1] = 0.0;
  const bool acoustic = k == 0 || k == NV - 1;
#pragma unroll
  for (int i = 0; i < NV; ++i) r[i] = acoustic ? ac[i] : (k == 1 ? en[i] : sh[i]);
}

template <int NV, int DIR, int W = -1, class Src>
__device__ __forceinline__ void lean_correction(const Src& src, unsigned mask, const FaceState<NV>& st,
                                                const KPhys& ph, double (&dF)[NV]) {
  double LF[NV], del[NV];
  project<NV, DIR>(st.s, st.Fc6, LF);
#define WL2_LF(K)                                                                            \
  if constexpr (K < NV) {                                                                    \
    del[K] = ((mask >> K) & 1u) ? lean_field<NV, DIR, K, W>(src, st.s, st.a[K], st.dv[K], LF[K], ph) \
                                : 0.0;                                                       \
  }
  WL2_LF(0) WL2_LF(1) WL2_LF(2) WL2_LF(3) WL2_LF(4)
#undef WL2_LF
  back_project<NV, DIR>(st.s, del, dF);
}

// The six stencil cells of the face of cell (x, y, z) along DIR below it
// (side 0) or above it (side 1) as light records, with the boundary ghosts
// (all loads issued before any use).
template <int NV, int DIR>
__device__ __forceinline__ void face_stencil(const double* U, const KGrid& g, const KPhys& ph, int x,
                                             int y, int z, int side, LRec<NV> (&w)[6]) {
  // the face below the cell starts 3 cells below it, the face above 2 below
  const int c0 = (DIR == 0 ? x : DIR == 1 ? y : z) + (side ? -2 : -3);
  double u[6][NV];
  bool flip[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int k = ghost_clamped(c0 + m, g.n[DIR], g.bc_lo[DIR], g.bc_hi[DIR], flip[m]);
    int p[3] = {x, y, z};
    p[DIR] = k;
    const long long off = p[0] + (long long)p[1] * g.stride[1] + (long long)p[2] * g.stride[2];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[m][v] = U[v * g.ncell + off];
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    if (flip[m]) u[m][1 + DIR] = -u[m][1 + DIR];
    if (DIR == 0 && c0 + m < 0 && g.bc_lo[0] == BC_INFLOW)
      load_inflow<NV>(g, y + (long long)g.n[1] * z, u[m]);
    if (DIR == 1 && NV == 4 && (c0 + m < 0 || c0 + m >= g.n[1]) && is_yghost(g, c0 + m))
      load_yghost<NV>(g, x, c0 + m, u[m]);
    make_lrec<NV>(u[m], ph, w[m]);
  }
}

// Nonlinear correction of one face of cell (x, y, z) along DIR: side 0 is
// the face below the cell, side 1 the face above.  Returns the change of the
// face flux (WENO minus linear, Eq.(33) per field).
template <int NV, int DIR, int SPLIT, int HYB, int W = -1>
__device__ __forceinline__ void face_delta(const double* U, const KGrid& g, const KPhys& ph,
                                           const unsigned long long* lfb, int x, int y, int z,
                                           int side, double (&dF)[NV]) {
  // the six stencil cells, kept in registers for the linear flux and every
  // field's correction
  LRec<NV> w[6];
  face_stencil<NV, DIR>(U, g, ph, x, y, z, side, w);
  const WinSrc<NV> src{w[0], w[1], w[2], w[3], w[4], w[5]};
  double Flin[NV];
  FaceState<NV> st;
  const unsigned mask = face_linear_st<NV, DIR, SPLIT, HYB>(src, ph, ph.eps_thr[DIR], lfb, Flin, st);
  if (mask) {
    lean_correction<NV, DIR, W>(src, mask, st, ph, dF);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) dF[v] = 0.0;
  }
}

// The same change of flux computed by NV lanes of one wavefront, lane k of
// them (the lanes lane0 .. lane0 + NV - 1, all active here) taking field k:
// each forms the linear face and the correction of its own field, and the
// lanes exchange those to back-project them.  Every lane ends with the bits
// face_delta gives (the same operations per field, summed alike).
template <int NV, int DIR, int SPLIT, int HYB, int W = -1>
__device__ __forceinline__ void face_delta_field(const double* U, const KGrid& g, const KPhys& ph,
                                                 const unsigned long long* lfb, int x, int y, int z,
                                                 int side, int k, int lane0, double (&dF)[NV]) {
  LRec<NV> w[6];
  face_stencil<NV, DIR>(U, g, ph, x, y, z, side, w);
  const WinSrc<NV> src{w[0], w[1], w[2], w[3], w[4], w[5]};
  double Flin[NV];
  FaceState<NV> st;
  const unsigned mask = face_linear_st<NV, DIR, SPLIT, HYB>(src, ph, ph.eps_thr[DIR], lfb, Flin, st);
  double LF[NV];
  project<NV, DIR>(st.s, st.Fc6, LF);
  double al = st.a[0], dvk = st.dv[0], LFk = LF[0];
#pragma unroll
  for (int j = 1; j < NV; ++j) {
    al = j == k ? st.a[j] : al;
    dvk = j == k ? st.dv[j] : dvk;
    LFk = j == k ? LF[j] : LFk;
  }
  double mine = 0.0;
  if ((mask >> k) & 1u) {
    double r[NV];
    left_row_rt<NV, DIR>(st.s, k, r);
    mine = lean_field_row<NV, DIR, W>(src, r, st.s, al, dvk, LFk, ph);
  }
  double del[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) del[j] = __shfl(mine, lane0 + j, 64);
  if (mask) {
    back_project<NV, DIR>(st.s, del, dF);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) dF[v] = 0.0;
  }
}

// Nonlinear correction of one listed cell by one lane: the flagged faces in
// the fixed order x-, x+, y-, y+, z-, z+, +dF for the face below the cell and
// -dF for the face above.
template <int NV, int SPLIT, int HYB, int W = -1>
__device__ __forceinline__ void serial_correction(const double* U, const KGrid& g,
                                                  const KPhys& ph, const StepCtl* ctl, int x,
                                                  int y, int z, unsigned cm, double (&acc)[NV]) {
  constexpr int NF = 2 * (NV - 2);
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int f = 0; f < NF; ++f) {
    if (!((cm >> f) & 1u)) continue;
    const int dir = f >> 1, side = f & 1;
    double dF[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) dF[v] = 0.0;
    if (dir == 0) {
      face_delta<NV, 0, SPLIT, HYB, W>(U, g, ph, ctl->lf_bits[0], x, y, z, side, dF);
    } else if (dir == 1) {
      if constexpr (NV >= 4)
        face_delta<NV, (NV >= 4 ? 1 : 0), SPLIT, HYB, W>(U, g, ph, ctl->lf_bits[1], x, y, z, side, dF);
    } else {
      if constexpr (NV >= 5)
        face_delta<NV, (NV >= 5 ? 2 : 0), SPLIT, HYB, W>(U, g, ph, ctl->lf_bits[2], x, y, z, side, dF);
    }
    const double sg = side ? -1.0 : 1.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += sg * dF[v];
  }
}

// Lanes given to a correction list in the one-lane-per-face mode: at most
// one wavefront per SIMD of the chip.  Lanes of one wavefront that take
// faces of different directions run one after the other, so per cell the
// grouped mode costs more lane-time than one lane per cell; it pays only
// while the list leaves the chip mostly idle.
constexpr unsigned long long FIX_GROUPED_LANES = 64ull * 1024ull;

// Nonlinear correction of one listed cell, computed by a group of GRP lanes
// of one wavefront: lane f of the group takes face f = 2 dir + side (x-, x+,
// y-, y+, z-, z+) if the mask flags it, and every lane of the group gets the
// sum of +-dF over the flagged faces in that fixed order (the face below the
// cell adds, the face above subtracts): the same bits as serial_correction,
// with one face of latency instead of six (for short lists; a long list
// keeps every lane busy with one cell each).
template <int NV, int GRP, int SPLIT, int HYB, int W = -1>
__device__ __forceinline__ void grouped_correction(const double* U, const KGrid& g,
                                                   const KPhys& ph, const StepCtl* ctl, int x,
                                                   int y, int z, unsigned cm, double (&acc)[NV]) {
  constexpr int NF = 2 * (NV - 2);
  static_assert(NF <= GRP && (64 % GRP) == 0, "one lane per face, groups inside a wavefront");
  const int lane = threadIdx.x & 63;
  const int f = lane % GRP;
  const int lane0 = lane - f;
  double dF[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) dF[v] = 0.0;
  if (f < NF && ((cm >> f) & 1u)) {
    const int dir = f >> 1, side = f & 1;
    if (dir == 0) {
      face_delta<NV, 0, SPLIT, HYB, W>(U, g, ph, ctl->lf_bits[0], x, y, z, side, dF);
    } else if (dir == 1) {
      if constexpr (NV >= 4)
        face_delta<NV, (NV >= 4 ? 1 : 0), SPLIT, HYB, W>(U, g, ph, ctl->lf_bits[1], x, y, z, side, dF);
    } else {
      if constexpr (NV >= 5)
        face_delta<NV, (NV >= 5 ? 2 : 0), SPLIT, HYB, W>(U, g, ph, ctl->lf_bits[2], x, y, z, side, dF);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
  for (int ff = 0; ff < NF; ++ff) {
    double d[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) d[v] = __shfl(dF[v], lane0 + ff, 64);
    if ((cm >> ff) & 1u) {
      const double sg = (ff & 1) ? -1.0 : 1.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += sg * d[v];
    }
  }
}

}  // namespace wl2
