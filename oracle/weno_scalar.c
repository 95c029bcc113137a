/*
 * Oracle (test infrastructure): scalar reconstruction of the incremental-
 * stencil WENO family.
 *
 * Follows Sec. 2.2, 2.4 and 3.1 of Zhu & Hu (arXiv 1908.02464):
 *   candidate fluxes of the four incremental-width stencils  Eq.(6)
 *   smoothness indicators beta_k and the reference tau_5      Eq.(11)
 *   L2-norm error terms E_k in closed form                    Eq.(27)
 *   weights, one of
 *     regularized weights alpha_k^r (the present scheme)      Eq.(28)
 *     original WENO-IS weights                                Eq.(8)
 *     WENO-IS with the 3-point indicator beta_01 of S01 on
 *     the two 2-point stencils (Wang et al.)                  Eq.(14)-(15)
 *   convex combination                                        Eq.(5)
 * Optimal weights d = (4,2,3,1)/10 as given after Eq.(8).
 */
#include "oracle_l2is.h"

double orc_weno_l2is(const double a[5], double lam, double eps_w, double *dbg) {
  return orc_weno(a, ORC_W_L2IS, lam, eps_w, dbg);
}

double orc_weno(const double a[5], int weights, double lam, double eps_w, double *dbg) {
  /* a[0..4] = f_{j-2}, f_{j-1}, f_j, f_{j+1}, f_{j+2} */
  const double fm2 = a[0], fm1 = a[1], f0 = a[2], fp1 = a[3], fp2 = a[4];
  const double d[4] = {4.0 / 10.0, 2.0 / 10.0, 3.0 / 10.0, 1.0 / 10.0};
  double q[4], beta[4], E[4], alpha[4], omega[4];
  double tau5, t1, t2, sum, fhat;
  int k;

  /* Eq.(6): candidate fluxes at x_{j+1/2} */
  q[0] = 0.5 * f0 + 0.5 * fp1;                                 /* S0 {j, j+1}     */
  q[1] = -0.5 * fm1 + 1.5 * f0;                                /* S1 {j-1, j}     */
  q[2] = f0 / 3.0 + 5.0 * fp1 / 6.0 - fp2 / 6.0;               /* S2 {j..j+2}     */
  q[3] = fm2 / 3.0 - 7.0 * fm1 / 6.0 + 11.0 * f0 / 6.0;        /* S3 {j-2..j}     */

  /* Eq.(11): smoothness indicators */
  beta[0] = (fp1 - f0) * (fp1 - f0);
  beta[1] = (f0 - fm1) * (f0 - fm1);
  t1 = f0 - 2.0 * fp1 + fp2;
  t2 = 3.0 * f0 - 4.0 * fp1 + fp2;
  beta[2] = 13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2;
  t1 = fm2 - 2.0 * fm1 + f0;
  t2 = fm2 - 4.0 * fm1 + 3.0 * f0;
  beta[3] = 13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2;
  t1 = fp2 - 4.0 * fp1 + 6.0 * f0 - 4.0 * fm1 + fm2;
  t2 = fp2 - 2.0 * fp1 + 2.0 * fm1 - fm2;
  tau5 = 13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2;

  /* Eq.(27): L2-norm error terms; the printed polynomial equals
   * (f_{j-1} - 2 f_j + f_{j+1})^2 / 45 for the two 2-point stencils. */
  t1 = fm1 - 2.0 * f0 + fp1;
  E[0] = t1 * t1 / 45.0;
  E[1] = E[0];
  E[2] = 0.0;
  E[3] = 0.0;

  sum = 0.0;
  if (weights == ORC_W_L2IS) {
    /* Eq.(28): regularized weights */
    for (k = 0; k < 4; ++k) {
      alpha[k] = d[k] * (1.0 + lam * tau5 / (lam * beta[k] + E[k] + eps_w));
      sum += alpha[k];
    }
  } else {
    /* Eq.(8): original WENO-IS weights (no lambda, no E_k) */
    double ratio[4];
    for (k = 0; k < 4; ++k) ratio[k] = tau5 / (beta[k] + eps_w);
    if (weights == ORC_W_IS_B01) {
      /* Eq.(15): smoothness indicator of the 3-point stencil S01 = {j-1,j,j+1};
       * Eq.(14): it multiplies the ratios of the two 2-point stencils */
      double b01, r01;
      t1 = fm1 - 2.0 * f0 + fp1;
      t2 = fm1 - fp1;
      b01 = 13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2;
      r01 = tau5 / (b01 + eps_w);
      ratio[0] *= r01;
      ratio[1] *= r01;
    }
    for (k = 0; k < 4; ++k) {
      alpha[k] = d[k] * (1.0 + ratio[k]);
      sum += alpha[k];
    }
  }
  fhat = 0.0;
  for (k = 0; k < 4; ++k) {
    omega[k] = alpha[k] / sum;
    fhat += omega[k] * q[k]; /* Eq.(5) */
  }

  if (dbg) {
    for (k = 0; k < 4; ++k) {
      dbg[k] = q[k];
      dbg[4 + k] = beta[k];
      dbg[9 + k] = E[k];
      dbg[13 + k] = omega[k];
    }
    dbg[8] = tau5;
  }
  return fhat;
}
