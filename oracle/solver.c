/*
 * Oracle (test infrastructure): grid-level semi-discretization and time
 * integration.
 *
 *   dU_j/dt = -(F_{j+1/2} - F_{j-1/2}) / dx, per direction, summed  Eq.(19)
 *   third-order TVD (SSP) Runge-Kutta in Shu-Osher form, CFL 0.5     Sec. 4
 *
 * Boundary ghosts (three layers per side, the paper names the conditions
 * only): periodic = wrap; transmissive = copy of the boundary cell;
 * reflective = mirror image of the interior with the normal momentum negated;
 * inflow (x- side of a 1D/2D grid, Sec. 4.7) = the prescribed state of the
 * x line, the same in all three ghosts.
 * The switch threshold of Eq.(35) uses L = thr_L[d] for direction d.
 * The time step is dt = cfl * dx / max_cells sum_d (|u_d| + c).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle_l2is.h"

typedef struct {
  int n[3], dim, nvar;
  long long ncell;
  double dx;  /* cell size (cell centres at (i + 1/2) dx): state ghosts */
} grid_t;

static int grid_init(grid_t *g, int nx, int ny, int nz) {
  if (nx < 1 || ny < 1 || nz < 1) return -1;
  if (nz > 1 && ny < 2) return -1;
  g->n[0] = nx;
  g->n[1] = ny;
  g->n[2] = nz;
  g->dim = nz > 1 ? 3 : (ny > 1 ? 2 : 1);
  g->nvar = g->dim + 2;
  g->ncell = (long long)nx * ny * nz;
  g->dx = 0.0;
  return 0;
}

static int check_params(const grid_t *g, const orc_params *p) {
  int d;
  for (d = 0; d < g->dim; ++d) {
    int lo = p->bc[2 * d], hi = p->bc[2 * d + 1];
    int slo = lo == ORC_BC_STATE_WALL || lo == ORC_BC_STATE_FRONT;
    int shi = hi == ORC_BC_STATE_WALL || hi == ORC_BC_STATE_FRONT;
    if (lo < 0 || lo > 5 || hi < 0 || hi > 5 || hi == ORC_BC_INFLOW) return -1;
    if ((slo || shi) && (d != 1 || g->dim != 2)) return -1;
    if (lo == ORC_BC_INFLOW && (d != 0 || g->dim == 3 || !p->inflow)) return -1;
    if ((lo == ORC_BC_PERIODIC) != (hi == ORC_BC_PERIODIC)) return -1;
    if ((lo == ORC_BC_REFLECTIVE || hi == ORC_BC_REFLECTIVE) && g->n[d] < 3) return -1;
    if (!(p->thr_L[d] > 0.0)) return -1;
  }
  if (p->split < 0 || p->split > 2 || p->hybrid < 0 || p->hybrid > 3) return -1;
  if (p->weights < ORC_W_L2IS || p->weights > ORC_W_IS_B01) return -1;
  return 0;
}

int orc_params_default(orc_params *p, int nx, int ny, int nz, double dx) {
  int d;
  p->cfl = 0.5;
  p->c_reg = 1.0;
  p->eps_w = 1e-20;
  p->thr_C = 1.0;
  p->thr_alpha = 3;
  p->split = ORC_SPLIT_LLF;
  p->hybrid = ORC_HYB_PER_FIELD;
  for (d = 0; d < 6; ++d) p->bc[d] = ORC_BC_TRANSMISSIVE;
  p->inflow = 0;
  p->weights = ORC_W_L2IS;
  memset(p->bstate, 0, sizeof(p->bstate));
  memset(p->bgeom, 0, sizeof(p->bgeom));
  p->time = 0.0;
  p->thr_L[0] = nx * dx;
  p->thr_L[1] = ny * dx;
  p->thr_L[2] = nz * dx;
  return 0;
}

static double threshold(const orc_params *p, double dx, int d) {
  double r = dx / p->thr_L[d], e = p->thr_C;
  int k;
  for (k = 0; k < p->thr_alpha; ++k) e *= r; /* C (dx/L)^alpha, Eq.(35) */
  return e;
}

/* Linear offset of cell (i0,i1,i2), component v. */
static long long at(const grid_t *g, int v, int i0, int i1, int i2) {
  return (((long long)v * g->n[2] + i2) * g->n[1] + i1) * g->n[0] + i0;
}

/* Interior index for line position k (may be outside 0..n-1) and whether the
 * normal momentum is negated (reflective ghost). */
static int ghost_map(int k, int n, int bclo, int bchi, int *flip) {
  *flip = 0;
  if (k >= 0 && k < n) return k;
  if (k < 0) {
    if (bclo == ORC_BC_PERIODIC) return ((k % n) + n) % n;
    if (bclo == ORC_BC_TRANSMISSIVE) return 0;
    if (bclo == ORC_BC_INFLOW) return -1; /* no interior source */
    *flip = 1;
    return -1 - k;
  }
  if (bchi == ORC_BC_PERIODIC) return k % n;
  if (bchi == ORC_BC_TRANSMISSIVE) return n - 1;
  *flip = 1;
  return 2 * n - 1 - k;
}

/* Component v of the state at cell idx of the line along d whose position
 * along d is k (a ghost when outside 0..n-1), boundary rules applied. */
static double cell_value(const grid_t *g, const orc_params *p, const double *U,
                         int d, int v, int k, const int idx[3]) {
  int flip, src;
  int i[3];
  double val;
  if (k < 0 || k >= g->n[d]) {
    /* state ghosts of a y side (2D): a prescribed state where the rule
     * gives one, else the mirror image of the interior */
    int kind = p->bc[2 * d + (k < 0 ? 0 : 1)];
    if (kind == ORC_BC_STATE_WALL || kind == ORC_BC_STATE_FRONT) {
      double xc = (idx[0] + 0.5) * g->dx, yc = (k + 0.5) * g->dx;
      if (kind == ORC_BC_STATE_FRONT)
        return xc < p->bgeom[1] + p->bgeom[2] * yc + p->bgeom[3] * p->time ? p->bstate[0][v]
                                                                          : p->bstate[1][v];
      if (xc < p->bgeom[0]) return p->bstate[0][v];
      src = k < 0 ? -1 - k : 2 * g->n[d] - 1 - k;
      i[0] = idx[0];
      i[1] = idx[1];
      i[2] = idx[2];
      i[d] = src;
      val = U[at(g, v, i[0], i[1], i[2])];
      return v == 1 + d ? -val : val;
    }
  }
  src = ghost_map(k, g->n[d], p->bc[2 * d], p->bc[2 * d + 1], &flip);
  if (src < 0) /* inflow ghost: the state given for this x line */
    return p->inflow[(long long)v * g->n[1] * g->n[2] + idx[1] + (long long)g->n[1] * idx[2]];
  i[0] = idx[0];
  i[1] = idx[1];
  i[2] = idx[2];
  i[d] = src;
  val = U[at(g, v, i[0], i[1], i[2])];
  return (flip && v == 1 + d) ? -val : val;
}

/* Gather the line through (c0,c1,c2) along d, with 3 ghosts per side,
 * into buf[(k+3)*nvar + v], k = -3..n+2. */
static void gather_line(const grid_t *g, const orc_params *p, const double *U,
                        int d, const int cidx[3], double *buf) {
  int n = g->n[d], k, v;
  for (k = -3; k < n + 3; ++k)
    for (v = 0; v < g->nvar; ++v) buf[(k + 3) * g->nvar + v] = cell_value(g, p, U, d, v, k, cidx);
}

/* Global LF speeds per field along d: max over cells of |lambda^s(U)|. */
static void lf_speeds(const grid_t *g, const double *U, double gamma, int d,
                      double *alpha) {
  long long c;
  int v, s;
  double u[5], F[5], prim[7];
  for (s = 0; s < g->nvar; ++s) alpha[s] = 0.0;
  for (c = 0; c < g->ncell; ++c) {
    for (v = 0; v < g->nvar; ++v) u[v] = U[v * g->ncell + c];
    orc_phys_flux(g->nvar, d, gamma, u, F, prim);
    for (s = 0; s < g->nvar; ++s) {
      double un = prim[1 + d], cs = prim[5];
      double e = fabs(s == 0 ? un - cs : (s == g->nvar - 1 ? un + cs : un));
      if (e > alpha[s]) alpha[s] = e;
    }
  }
}

/* Face fluxes along one line: Fl[f*nvar + v], f = 0..n (face f between cells
 * f-1 and f). */
static int line_fluxes(const grid_t *g, const orc_params *p, double gamma,
                       double eps_thr, const double *alpha_lf, int d,
                       const double *buf, double *Fl, unsigned char *fl,
                       double *sg) {
  int n = g->n[d], f, rc;
  for (f = 0; f <= n; ++f) {
    /* cells f-3 .. f+2 are buf rows f .. f+5 */
    rc = orc_face_flux(g->nvar, d, gamma, p, eps_thr, alpha_lf,
                       buf + f * g->nvar, Fl + f * g->nvar,
                       fl ? fl + f * g->nvar : 0, sg ? sg + f * g->nvar : 0);
    if (rc) return rc;
  }
  return 0;
}

/* Enumerate the lines along d: the two other indices. */
static void line_index(const grid_t *g, int d, long long line, int cidx[3]) {
  int a = (d == 0) ? 1 : 0, b = (d == 2) ? 1 : 2;
  cidx[d] = 0;
  cidx[a] = (int)(line % g->n[a]);
  cidx[b] = (int)(line / g->n[a]);
}

static int add_direction(const grid_t *g, const orc_params *p, double gamma,
                         double dx, int d, const double *U, double *dUdt) {
  int n = g->n[d], rc = 0;
  long long nlines = g->ncell / n;
  double eps_thr = threshold(p, dx, d), alpha_lf[5];
  if (p->split == ORC_SPLIT_LF) lf_speeds(g, U, gamma, d, alpha_lf);
  /* lines are independent (each writes only its own cells), so a build with
   * OpenMP may hand them to threads: the result does not depend on how many */
#pragma omp parallel
  {
    long long line;
    int i, v, lrc = 0;
    double *buf = (double *)malloc(sizeof(double) * (n + 6) * g->nvar);
    double *Fl = (double *)malloc(sizeof(double) * (n + 1) * g->nvar);
    if (!buf || !Fl) lrc = -2;
#pragma omp for schedule(static)
    for (line = 0; line < nlines; ++line) {
      int cidx[3];
      if (lrc) continue;
      line_index(g, d, line, cidx);
      gather_line(g, p, U, d, cidx, buf);
      lrc = line_fluxes(g, p, gamma, eps_thr, alpha_lf, d, buf, Fl, 0, 0);
      for (i = 0; i < n && !lrc; ++i) {
        int idx[3];
        idx[0] = cidx[0];
        idx[1] = cidx[1];
        idx[2] = cidx[2];
        idx[d] = i;
        for (v = 0; v < g->nvar; ++v)
          dUdt[at(g, v, idx[0], idx[1], idx[2])] -=
              (Fl[(i + 1) * g->nvar + v] - Fl[i * g->nvar + v]) / dx;
      }
    }
#pragma omp critical
    if (lrc && !rc) rc = lrc;
    free(buf);
    free(Fl);
  }
  return rc;
}

int orc_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int orc_rhs(const double *U, int nx, int ny, int nz, double dx, double gamma,
            const orc_params *p, double *dUdt) {
  grid_t g;
  int d, rc;
  long long k;
  if (!U || !dUdt || !p || !(dx > 0.0) || !(gamma > 1.0)) return -1;
  if (grid_init(&g, nx, ny, nz) || check_params(&g, p)) return -1;
  g.dx = dx;
  for (k = 0; k < g.ncell * g.nvar; ++k) dUdt[k] = 0.0;
  for (d = 0; d < g.dim; ++d) {
    rc = add_direction(&g, p, gamma, dx, d, U, dUdt);
    if (rc) return rc;
  }
  return 0;
}

int orc_rhs_at(const double *U, int nx, int ny, int nz, double dx,
               double gamma, const orc_params *p, int ncells,
               const long long *cell, double *out) {
  grid_t g;
  int d, v, q, rc;
  double buf[12 * 5], Fl[2 * 5], alpha_lf[3][5];
  if (!U || !out || !p || !cell || ncells < 0 || !(dx > 0.0) || !(gamma > 1.0))
    return -1;
  if (grid_init(&g, nx, ny, nz) || check_params(&g, p)) return -1;
  g.dx = dx;
  if (p->split == ORC_SPLIT_LF)
    for (d = 0; d < g.dim; ++d) lf_speeds(&g, U, gamma, d, alpha_lf[d]);
  for (q = 0; q < ncells; ++q) {
    long long c = cell[q];
    int ci[3];
    if (c < 0 || c >= g.ncell) return -1;
    ci[0] = (int)(c % nx);
    ci[1] = (int)((c / nx) % ny);
    ci[2] = (int)(c / ((long long)nx * ny));
    for (v = 0; v < g.nvar; ++v) out[v * ncells + q] = 0.0;
    for (d = 0; d < g.dim; ++d) {
      /* cells i-3 .. i+3 around the target along d, ghosts applied */
      int k;
      double eps_thr = threshold(p, dx, d);
      for (k = -3; k <= 3; ++k)
        for (v = 0; v < g.nvar; ++v)
          buf[(k + 3) * g.nvar + v] = cell_value(&g, p, U, d, v, ci[d] + k, ci);
      /* face i-1/2 uses cells i-3..i+2, face i+1/2 uses i-2..i+3 */
      rc = orc_face_flux(g.nvar, d, gamma, p, eps_thr, alpha_lf[d], buf, Fl, 0, 0);
      if (rc) return rc;
      rc = orc_face_flux(g.nvar, d, gamma, p, eps_thr, alpha_lf[d],
                         buf + g.nvar, Fl + g.nvar, 0, 0);
      if (rc) return rc;
      for (v = 0; v < g.nvar; ++v)
        out[v * ncells + q] -= (Fl[g.nvar + v] - Fl[v]) / dx;
    }
  }
  return 0;
}

int orc_face_debug(const double *U, int nx, int ny, int nz, double dx,
                   double gamma, const orc_params *p, int d,
                   unsigned char *flags, double *sigma) {
  grid_t g;
  int n, f, v, s, rc = 0;
  long long nlines, line, nface;
  double eps_thr, alpha_lf[5], *buf, *Fl, *sg;
  unsigned char *fl;
  int fn[3];
  if (!U || !flags || !sigma || !p || !(dx > 0.0) || !(gamma > 1.0)) return -1;
  if (grid_init(&g, nx, ny, nz) || check_params(&g, p)) return -1;
  g.dx = dx;
  if (d < 0 || d >= g.dim) return -1;
  n = g.n[d];
  nlines = g.ncell / n;
  fn[0] = g.n[0];
  fn[1] = g.n[1];
  fn[2] = g.n[2];
  fn[d] = n + 1;
  nface = (long long)fn[0] * fn[1] * fn[2];
  eps_thr = threshold(p, dx, d);
  if (p->split == ORC_SPLIT_LF) lf_speeds(&g, U, gamma, d, alpha_lf);
  buf = (double *)malloc(sizeof(double) * (n + 6) * g.nvar);
  Fl = (double *)malloc(sizeof(double) * (n + 1) * g.nvar);
  sg = (double *)malloc(sizeof(double) * (n + 1) * g.nvar);
  fl = (unsigned char *)malloc((size_t)(n + 1) * g.nvar);
  if (!buf || !Fl || !sg || !fl) rc = -2;
  for (line = 0; line < nlines && !rc; ++line) {
    int cidx[3];
    line_index(&g, d, line, cidx);
    gather_line(&g, p, U, d, cidx, buf);
    rc = line_fluxes(&g, p, gamma, eps_thr, alpha_lf, d, buf, Fl, fl, sg);
    for (f = 0; f <= n && !rc; ++f) {
      int idx[3];
      long long o;
      idx[0] = cidx[0];
      idx[1] = cidx[1];
      idx[2] = cidx[2];
      idx[d] = f;
      o = ((long long)idx[2] * fn[1] + idx[1]) * fn[0] + idx[0];
      for (s = 0; s < g.nvar; ++s) {
        flags[s * nface + o] = fl[f * g.nvar + s];
        sigma[s * nface + o] = sg[f * g.nvar + s];
      }
    }
  }
  (void)v;
  free(buf);
  free(Fl);
  free(sg);
  free(fl);
  return rc;
}

static int nonphysical(const grid_t *g, const double *U, double gamma, long long c) {
  int v, k;
  double rho = U[c], E = U[(g->nvar - 1) * g->ncell + c], q = 0.0, pr;
  for (v = 0; v < g->nvar; ++v)
    if (!isfinite(U[v * g->ncell + c])) return 1;
  if (!(rho > 0.0)) return 1;
  for (k = 0; k < g->dim; ++k) {
    double u = U[(1 + k) * g->ncell + c] / rho;
    q += u * u;
  }
  pr = (gamma - 1.0) * (E - rho * 0.5 * q);
  return !(pr > 0.0);
}

/* max over the cells of sum_d (|u_d| + c) (NaN if a cell gives NaN);
 * *bad set when a cell is non-physical. */
static double interior_speed(const grid_t *g, const double *U, double gamma, int *bad) {
  long long c;
  int v, d;
  double smax = 0.0, u[5], F[5], prim[7];
  *bad = 0;
  for (c = 0; c < g->ncell; ++c) {
    double s = 0.0;
    if (nonphysical(g, U, gamma, c)) *bad = 1;
    for (v = 0; v < g->nvar; ++v) u[v] = U[v * g->ncell + c];
    orc_phys_flux(g->nvar, 0, gamma, u, F, prim);
    for (d = 0; d < g->dim; ++d) s += fabs(prim[1 + d]) + prim[5];
    if (s > smax || s != s) smax = s;
  }
  return smax;
}

int orc_cfl_dt(const double *U, int nx, int ny, int nz, double dx,
               double gamma, double cfl, double *dt) {
  grid_t g;
  int bad;
  double smax;
  if (!U || !dt || !(dx > 0.0) || !(gamma > 1.0) || !(cfl > 0.0)) return -1;
  if (grid_init(&g, nx, ny, nz)) return -1;
  smax = interior_speed(&g, U, gamma, &bad);
  *dt = cfl * dx / smax;
  return bad;
}

/* Time step of the scheme: the CFL step of the interior, with the speed of
 * the inflow ghost states included when the x- side is an inflow (the jet
 * enters at its own speed, which no interior cell has at the start). */
static int scheme_dt(const double *U, const grid_t *g, double dx, double gamma,
                     const orc_params *p, double *dt) {
  int st;
  double smax = interior_speed(g, U, gamma, &st);
  if (p->bc[0] == ORC_BC_INFLOW) {
    long long rows = (long long)g->n[1] * g->n[2], r;
    double u[5], F[5], prim[7];
    int v, d;
    for (r = 0; r < rows; ++r) {
      double s = 0.0;
      for (v = 0; v < g->nvar; ++v) u[v] = p->inflow[v * rows + r];
      orc_phys_flux(g->nvar, 0, gamma, u, F, prim);
      for (d = 0; d < g->dim; ++d) s += fabs(prim[1 + d]) + prim[5];
      if (s > smax) smax = s;
    }
  }
  *dt = p->cfl * dx / smax;
  return st;
}

int orc_step(double *U, int nx, int ny, int nz, double dx, double gamma,
             const orc_params *p, double dt_in, double *dt_used) {
  grid_t g;
  long long k, N;
  double dt, *U1, *U2, *Lk;
  int rc, st = 0;
  orc_params ps;
  if (!U || !p || !(dx > 0.0) || !(gamma > 1.0)) return -1;
  if (grid_init(&g, nx, ny, nz) || check_params(&g, p)) return -1;
  N = g.ncell * g.nvar;
  if (dt_in > 0.0) {
    dt = dt_in;
  } else {
    st = scheme_dt(U, &g, dx, gamma, p, &dt);
    if (st < 0) return st;
  }
  if (dt_used) *dt_used = dt;
  U1 = (double *)malloc(sizeof(double) * N);
  U2 = (double *)malloc(sizeof(double) * N);
  Lk = (double *)malloc(sizeof(double) * N);
  if (!U1 || !U2 || !Lk) {
    free(U1);
    free(U2);
    free(Lk);
    return -2;
  }
  ps = *p; /* the stages' own times: t, t + dt, t + dt/2 */
  /* U1 = U + dt L(U) */
  rc = orc_rhs(U, nx, ny, nz, dx, gamma, &ps, Lk);
  for (k = 0; k < N && !rc; ++k) U1[k] = U[k] + dt * Lk[k];
  /* U2 = 3/4 U + 1/4 (U1 + dt L(U1)) */
  ps.time = p->time + dt;
  if (!rc) rc = orc_rhs(U1, nx, ny, nz, dx, gamma, &ps, Lk);
  for (k = 0; k < N && !rc; ++k) U2[k] = 0.75 * U[k] + 0.25 * (U1[k] + dt * Lk[k]);
  /* U = 1/3 U + 2/3 (U2 + dt L(U2)) */
  ps.time = p->time + 0.5 * dt;
  if (!rc) rc = orc_rhs(U2, nx, ny, nz, dx, gamma, &ps, Lk);
  for (k = 0; k < N && !rc; ++k)
    U[k] = (1.0 / 3.0) * U[k] + (2.0 / 3.0) * (U2[k] + dt * Lk[k]);
  free(U1);
  free(U2);
  free(Lk);
  if (rc) return rc;
  return st;
}

int orc_run(double *U, int nx, int ny, int nz, double dx, double gamma,
            const orc_params *p, double t_end, int max_steps, double *t_out,
            int *steps_out) {
  double t, dt;
  int steps = 0, st = 0;
  grid_t g;
  orc_params pt;
  if (!U || !p || !(dx > 0.0) || !(gamma > 1.0)) return -1;
  if (grid_init(&g, nx, ny, nz) || check_params(&g, p)) return -1;
  pt = *p;
  t = p->time;
  while (t < t_end && steps < max_steps) {
    st = scheme_dt(U, &g, dx, gamma, p, &dt);
    if (st) break;
    if (t + dt > t_end) dt = t_end - t;
    pt.time = t;
    st = orc_step(U, nx, ny, nz, dx, gamma, &pt, dt, 0);
    if (st) break;
    t += dt;
    ++steps;
  }
  if (!st) {
    double dtx;
    st = orc_cfl_dt(U, nx, ny, nz, dx, gamma, p->cfl, &dtx);
  }
  if (t_out) *t_out = t;
  if (steps_out) *steps_out = steps;
  return st;
}
