/*
 * Oracle (test infrastructure): Euler physics and the characteristic system.
 *
 *   ideal-gas Euler equations and their flux              Eq.(17)-(18)
 *   Roe average at x_{j+1/2}                               Sec. 2.3, step (1)
 *   left/right eigenvectors and eigenvalues of the
 *   Roe-averaged Jacobian                                  Sec. 2.3, step (2)
 *
 * The paper states the 1D system only; the 2D/3D systems are treated
 * dimension by dimension, the sweep direction's momentum taking the role of
 * the 1D momentum and each tangential momentum adding one shear field.
 *
 * Eigenvector scaling (the paper leaves it open): acoustic and entropy
 * right eigenvectors have unit density component; shear right eigenvectors
 * are scaled by the Roe sound speed.  Every characteristic variable L^s . U
 * then carries density units, which the detector of Eq.(30) divides by the
 * Roe density to make non-dimensional.
 */
#include <math.h>
#include "oracle_l2is.h"

static int dim_of(int nvar) { return nvar - 2; }

int orc_phys_flux(int nvar, int dir, double gamma, const double *U, double *F,
                  double *prim) {
  int dim = dim_of(nvar), k;
  double rho, vel[3] = {0.0, 0.0, 0.0}, E, q, p, c, H;
  if (dim < 1 || dim > 3 || dir < 0 || dir >= dim) return -1;
  rho = U[0];
  E = U[nvar - 1];
  for (k = 0; k < dim; ++k) vel[k] = U[1 + k] / rho;
  q = 0.0;
  for (k = 0; k < dim; ++k) q += vel[k] * vel[k];
  q *= 0.5;
  p = (gamma - 1.0) * (E - rho * q); /* E = p/(gamma-1) + rho |u|^2 / 2 */
  c = sqrt(gamma * p / rho);
  H = (E + p) / rho;
  /* F_d(U) = (rho u_d, rho u_d u + p e_d, (E + p) u_d) */
  F[0] = U[1 + dir];
  for (k = 0; k < dim; ++k) F[1 + k] = U[1 + dir] * vel[k] + (k == dir ? p : 0.0);
  F[nvar - 1] = (E + p) * vel[dir];
  if (prim) {
    prim[0] = rho;
    prim[1] = vel[0];
    prim[2] = vel[1];
    prim[3] = vel[2];
    prim[4] = p;
    prim[5] = c;
    prim[6] = H;
  }
  return 0;
}

int orc_roe_eigen(int nvar, int dir, double gamma, const double *UL,
                  const double *UR, double *L, double *R, double *lam,
                  double *roe) {
  int dim = dim_of(nvar), k, i, s;
  double FL[5], FR[5], pl[7], pr[7];
  double wl, wr, ut[3] = {0.0, 0.0, 0.0}, Ht, rhot, qt, ct, b1, b2, un;
  int tang[2], ntang = 0;
  if (dim < 1 || dim > 3 || dir < 0 || dir >= dim) return -1;
  orc_phys_flux(nvar, dir, gamma, UL, FL, pl);
  orc_phys_flux(nvar, dir, gamma, UR, FR, pr);

  /* Roe average with sqrt(rho) weights */
  wl = sqrt(pl[0]);
  wr = sqrt(pr[0]);
  for (k = 0; k < dim; ++k) ut[k] = (wl * pl[1 + k] + wr * pr[1 + k]) / (wl + wr);
  Ht = (wl * pl[6] + wr * pr[6]) / (wl + wr);
  rhot = wl * wr; /* Roe density sqrt(rho_L rho_R), used by Eq.(30) */
  qt = 0.0;
  for (k = 0; k < dim; ++k) qt += ut[k] * ut[k];
  qt *= 0.5;
  ct = sqrt((gamma - 1.0) * (Ht - qt));
  un = ut[dir];
  b1 = (gamma - 1.0) / (ct * ct);
  b2 = b1 * qt;

  for (k = 0; k < dim; ++k)
    if (k != dir) tang[ntang++] = k;

  for (i = 0; i < nvar * nvar; ++i) {
    L[i] = 0.0;
    R[i] = 0.0;
  }
  /* columns of R (R[i*nvar + s]) and rows of L (L[s*nvar + i]) */
  /* s = 0 : u_n - c */
  s = 0;
  R[0 * nvar + s] = 1.0;
  for (k = 0; k < dim; ++k) R[(1 + k) * nvar + s] = ut[k] - (k == dir ? ct : 0.0);
  R[(nvar - 1) * nvar + s] = Ht - un * ct;
  L[s * nvar + 0] = 0.5 * (b2 + un / ct);
  for (k = 0; k < dim; ++k)
    L[s * nvar + 1 + k] = 0.5 * (-b1 * ut[k] - (k == dir ? 1.0 / ct : 0.0));
  L[s * nvar + nvar - 1] = 0.5 * b1;
  /* s = 1 : entropy wave u_n */
  s = 1;
  R[0 * nvar + s] = 1.0;
  for (k = 0; k < dim; ++k) R[(1 + k) * nvar + s] = ut[k];
  R[(nvar - 1) * nvar + s] = qt;
  L[s * nvar + 0] = 1.0 - b2;
  for (k = 0; k < dim; ++k) L[s * nvar + 1 + k] = b1 * ut[k];
  L[s * nvar + nvar - 1] = -b1;
  /* shear waves u_n, one per tangential direction */
  for (i = 0; i < ntang; ++i) {
    int t = tang[i];
    s = 2 + i;
    R[(1 + t) * nvar + s] = ct;
    R[(nvar - 1) * nvar + s] = ct * ut[t];
    L[s * nvar + 0] = -ut[t] / ct;
    L[s * nvar + 1 + t] = 1.0 / ct;
  }
  /* s = nvar-1 : u_n + c */
  s = nvar - 1;
  R[0 * nvar + s] = 1.0;
  for (k = 0; k < dim; ++k) R[(1 + k) * nvar + s] = ut[k] + (k == dir ? ct : 0.0);
  R[(nvar - 1) * nvar + s] = Ht + un * ct;
  L[s * nvar + 0] = 0.5 * (b2 - un / ct);
  for (k = 0; k < dim; ++k)
    L[s * nvar + 1 + k] = 0.5 * (-b1 * ut[k] + (k == dir ? 1.0 / ct : 0.0));
  L[s * nvar + nvar - 1] = 0.5 * b1;

  if (lam) {
    lam[0] = un - ct;
    for (s = 1; s < nvar - 1; ++s) lam[s] = un;
    lam[nvar - 1] = un + ct;
  }
  if (roe) {
    roe[0] = rhot;
    roe[1] = ut[0];
    roe[2] = ut[1];
    roe[3] = ut[2];
    roe[4] = Ht;
    roe[5] = ct;
  }
  return 0;
}
