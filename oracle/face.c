/*
 * Oracle (test infrastructure): the numerical flux at one face x_{j+1/2}.
 *
 * Steps, in the paper's order (Sec. 2.3 and Sec. 3.2-3.3):
 *   (1)-(2) Roe average and eigensystem                 (charsys.c)
 *   detector  dv^s = L^s . (U_{j-2} - 5U_{j-1} + 10U_j - 10U_{j+1}
 *                           + 5U_{j+2} - U_{j+3}) / 60   Eq.(31)
 *             sigma^s = (dv^s / rho~)^2                  Eq.(30)
 *   regularization parameter lambda = c sigma^s         Eq.(32)
 *   switch: sigma^s < eps -> optimal linear scheme       Eq.(33),(35)
 *   linear flux, per field:
 *      L^s . (F_{j-2} - 8F_{j-1} + 37F_j + 37F_{j+1} - 8F_{j+2} + F_{j+3})/60
 *      + alpha^s dv^s                                    Eq.(34)
 *     (the dissipation term of Eq.(34) read with the 1/60 applied and the
 *      splitting speed alpha^s: exactly the d-weighted upwind combination of
 *      the split fluxes below)
 *   WENO flux, per field:
 *      (3) v_m = L^s . U_m, g_m = L^s . F_m, m = j-2..j+3     Eq.(20)
 *      (4) f^{s,+-}_m = (g_m +- alpha^s v_m) / 2               Eq.(21)
 *      (5) f+ from (f+_{j-2..j+2}); f- by mirror symmetry about x_{j+1/2},
 *          i.e. the same routine on (f-_{j+3}, ..., f-_{j-1})  Eq.(22)
 *          f^s = f+ + f-                                       Eq.(23)
 *   (6) back projection F = sum_s R^s f^s                      Eq.(24)
 * Splitting speed alpha^s (Eq.(21)): LLF = max over the six stencil cells of
 * the cell eigenvalue |lambda^s(U_m)|; LF = supplied global maximum;
 * Roe = |lambda^s| of the Roe-averaged Jacobian.
 */
#include <math.h>
#include "oracle_l2is.h"

static double cell_eig(int nvar, int s, const double *prim, int dir) {
  double un = prim[1 + dir], c = prim[5];
  if (s == 0) return un - c;
  if (s == nvar - 1) return un + c;
  return un;
}

int orc_face_flux(int nvar, int dir, double gamma, const orc_params *p,
                  double eps_thr, const double *alpha_lf, const double *U6,
                  double *Fhat, unsigned char *flags, double *sigma) {
  double L[25], R[25], lam[5], roe[6];
  double F6[6][5], prim6[6][7], dU5[5], Fc6[5];
  double dv[5], sig[5], alpha[5], fs[5];
  unsigned char lin[5];
  int i, s, m, rc;
  const double *Um[6];

  for (m = 0; m < 6; ++m) {
    Um[m] = U6 + m * nvar;
    rc = orc_phys_flux(nvar, dir, gamma, Um[m], F6[m], prim6[m]);
    if (rc) return rc;
  }
  /* steps (1)-(2): cells j (m=2) and j+1 (m=3) */
  rc = orc_roe_eigen(nvar, dir, gamma, Um[2], Um[3], L, R, lam, roe);
  if (rc) return rc;

  /* fifth difference of U and the six-point central flux, with symmetric
   * pairing of the stencil points */
  for (i = 0; i < nvar; ++i) {
    dU5[i] = (Um[0][i] - Um[5][i]) + 5.0 * (Um[4][i] - Um[1][i]) +
             10.0 * (Um[2][i] - Um[3][i]);
    Fc6[i] = ((F6[0][i] + F6[5][i]) - 8.0 * (F6[1][i] + F6[4][i]) +
              37.0 * (F6[2][i] + F6[3][i])) / 60.0;
  }

  for (s = 0; s < nvar; ++s) {
    double acc = 0.0;
    for (i = 0; i < nvar; ++i) acc += L[s * nvar + i] * dU5[i];
    dv[s] = acc / 60.0;                                   /* Eq.(31) */
    sig[s] = (dv[s] / roe[0]) * (dv[s] / roe[0]);         /* Eq.(30) */
    if (p->split == ORC_SPLIT_LLF) {
      double a = 0.0;
      for (m = 0; m < 6; ++m) {
        double e = fabs(cell_eig(nvar, s, prim6[m], dir));
        if (e > a) a = e;
      }
      alpha[s] = a;
    } else if (p->split == ORC_SPLIT_LF) {
      alpha[s] = alpha_lf[s];
    } else {
      alpha[s] = fabs(lam[s]);
    }
  }

  /* switch of Eq.(33)/(35) */
  {
    double smax = 0.0;
    for (s = 0; s < nvar; ++s)
      if (sig[s] > smax || sig[s] != sig[s]) smax = sig[s];
    for (s = 0; s < nvar; ++s) {
      switch (p->hybrid) {
        case ORC_HYB_PER_FACE: lin[s] = (unsigned char)(smax < eps_thr); break;
        case ORC_HYB_WENO_ONLY: lin[s] = 0; break;
        case ORC_HYB_LINEAR_ONLY: lin[s] = 1; break;
        default: lin[s] = (unsigned char)(sig[s] < eps_thr); break;
      }
    }
  }

  for (s = 0; s < nvar; ++s) {
    if (lin[s]) {
      double acc = 0.0;
      for (i = 0; i < nvar; ++i) acc += L[s * nvar + i] * Fc6[i];
      fs[s] = acc + alpha[s] * dv[s];                     /* Eq.(34) */
    } else {
      double v[6], g[6], fp[6], fm[6], ap[5], am[5], lr;
      for (m = 0; m < 6; ++m) {
        double av = 0.0, ag = 0.0;
        for (i = 0; i < nvar; ++i) {
          av += L[s * nvar + i] * Um[m][i];
          ag += L[s * nvar + i] * F6[m][i];
        }
        v[m] = av;                                        /* Eq.(20) */
        g[m] = ag;
        fp[m] = 0.5 * (g[m] + alpha[s] * v[m]);           /* Eq.(21) */
        fm[m] = 0.5 * (g[m] - alpha[s] * v[m]);
      }
      lr = p->c_reg * sig[s];                             /* Eq.(32) */
      for (m = 0; m < 5; ++m) {
        ap[m] = fp[m];          /* f+_{j-2} .. f+_{j+2} */
        am[m] = fm[5 - m];      /* f-_{j+3} .. f-_{j-1} (mirrored) */
      }
      fs[s] = orc_weno(ap, p->weights, lr, p->eps_w, 0) +
              orc_weno(am, p->weights, lr, p->eps_w, 0);  /* Eq.(22)-(23) */
    }
  }

  for (i = 0; i < nvar; ++i) {
    double acc = 0.0;
    for (s = 0; s < nvar; ++s) acc += R[i * nvar + s] * fs[s]; /* Eq.(24) */
    Fhat[i] = acc;
  }
  if (flags)
    for (s = 0; s < nvar; ++s) flags[s] = lin[s];
  if (sigma)
    for (s = 0; s < nvar; ++s) sigma[s] = sig[s];
  return 0;
}
