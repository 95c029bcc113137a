/*
 * Host driver for the oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built and run by test_oracle_sanitizers.py):
 * every entry point of oracle_l2is.h on small 1D, 2D and 3D grids with
 * every boundary kind, splitting, switch mode and weighting, and the
 * refusals of invalid arguments.  Any out-of-bounds access, use after free,
 * leak or undefined operation aborts the run; a wrong return code exits 1.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_l2is.h"

static unsigned long long rng_state = 88172645463325252ull;

/* xorshift64 (Marsaglia), uniform in [0, 1) */
static double urand(void) {
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static void rand_state(int nvar, double *u) {
  int dim = nvar - 2, k;
  double rho = 0.5 + urand(), p = 0.5 + urand(), ke = 0.0;
  u[0] = rho;
  for (k = 0; k < dim; ++k) {
    double v = urand() - 0.5;
    u[1 + k] = rho * v;
    ke += 0.5 * rho * v * v;
  }
  u[nvar - 1] = p / 0.4 + ke;
}

static int failures = 0;

static void expect(int cond, const char *what) {
  if (!cond) {
    fprintf(stderr, "unexpected result: %s\n", what);
    ++failures;
  }
}

static void grid_case(int nx, int ny, int nz, const int bc[6], int split, int hybrid,
                      int weights) {
  const int dim = nz > 1 ? 3 : (ny > 1 ? 2 : 1);
  const int nvar = dim + 2;
  const long long nc = (long long)nx * ny * nz;
  const double dx = 0.1, gamma = 1.4;
  double *U = malloc(sizeof(double) * nvar * nc);
  double *out = malloc(sizeof(double) * nvar * nc);
  double *inflow = malloc(sizeof(double) * nvar * ny * nz);
  double u[5];
  long long c, cells[3];
  int v, d, st, steps;
  double dt, t;
  orc_params p;
  for (c = 0; c < nc; ++c) {
    rand_state(nvar, u);
    for (v = 0; v < nvar; ++v) U[v * nc + c] = u[v];
  }
  for (c = 0; c < (long long)ny * nz; ++c) {
    rand_state(nvar, u);
    for (v = 0; v < nvar; ++v) inflow[v * ny * nz + c] = u[v];
  }
  expect(orc_params_default(&p, nx, ny, nz, dx) == 0, "params_default");
  memcpy(p.bc, bc, sizeof(p.bc));
  p.split = split;
  p.hybrid = hybrid;
  p.weights = weights;
  p.inflow = bc[0] == ORC_BC_INFLOW ? inflow : NULL;
  for (v = 0; v < 2; ++v) rand_state(nvar, p.bstate[v]);
  p.bgeom[0] = 0.3;
  p.bgeom[1] = 0.2;
  p.bgeom[2] = 0.5;
  p.bgeom[3] = 2.0;
  p.time = 0.01;
  expect(orc_rhs(U, nx, ny, nz, dx, gamma, &p, out) == 0, "rhs");
  cells[0] = 0;
  cells[1] = nc / 2;
  cells[2] = nc - 1;
  expect(orc_rhs_at(U, nx, ny, nz, dx, gamma, &p, 3, cells, out) == 0, "rhs_at");
  for (d = 0; d < dim; ++d) {
    long long nf = nc / (d == 0 ? nx : d == 1 ? ny : nz) * ((d == 0 ? nx : d == 1 ? ny : nz) + 1);
    unsigned char *fl = malloc((size_t)nvar * nf);
    double *sg = malloc(sizeof(double) * nvar * nf);
    expect(orc_face_debug(U, nx, ny, nz, dx, gamma, &p, d, fl, sg) == 0, "face_debug");
    free(fl);
    free(sg);
  }
  expect(orc_cfl_dt(U, nx, ny, nz, dx, gamma, 0.5, &dt) == 0, "cfl_dt");
  st = orc_step(U, nx, ny, nz, dx, gamma, &p, 0.0, &dt);
  expect(st == 0 || st == 1, "step");
  st = orc_run(U, nx, ny, nz, dx, gamma, &p, p.time + 10.0, 3, &t, &steps);
  expect(st == 0 || st == 1, "run");
  free(U);
  free(out);
  free(inflow);
}

int main(void) {
  int nvar, dir, s, h, w, k;
  double a[5], dbg[17], U6[30], F[5], sg[5], L[25], R[25], lam[5], roe[6], prim[7];
  unsigned char fl[5];
  orc_params p;
  orc_threads(1);
  /* scalar reconstructions and the face flux */
  for (k = 0; k < 50; ++k) {
    for (s = 0; s < 5; ++s) a[s] = urand() - 0.5;
    for (w = 0; w < 3; ++w) (void)orc_weno(a, w, urand(), 1e-20, dbg);
    (void)orc_weno_l2is(a, urand(), 1e-20, NULL);
  }
  for (nvar = 3; nvar <= 5; ++nvar) {
    for (dir = 0; dir < nvar - 2; ++dir) {
      double alf[5] = {3.0, 3.0, 3.0, 3.0, 3.0};
      for (k = 0; k < 6; ++k) rand_state(nvar, U6 + k * nvar);
      expect(orc_roe_eigen(nvar, dir, 1.4, U6, U6 + nvar, L, R, lam, roe) == 0, "roe_eigen");
      expect(orc_phys_flux(nvar, dir, 1.4, U6, F, prim) == 0, "phys_flux");
      orc_params_default(&p, 8, 1, 1, 0.1);
      for (s = 0; s < 3; ++s)
        for (h = 0; h < 4; ++h)
          for (w = 0; w < 3; ++w) {
            p.split = s;
            p.hybrid = h;
            p.weights = w;
            expect(orc_face_flux(nvar, dir, 1.4, &p, 1e-6, alf, U6, F, fl, sg) == 0, "face_flux");
          }
    }
  }
  /* grids: every boundary kind in the dimensions that define it */
  {
    const int per[6] = {0, 0, 0, 0, 0, 0}, tra[6] = {1, 1, 1, 1, 1, 1};
    const int ref[6] = {2, 2, 2, 2, 2, 2}, mix[6] = {0, 0, 2, 1, 1, 2};
    const int inf[6] = {3, 1, 2, 1, 1, 1}, dmr[6] = {3, 1, 4, 5, 1, 1};
    const int *sets[6] = {per, tra, ref, mix, inf, dmr};
    const int shapes[3][3] = {{13, 1, 1}, {11, 9, 1}, {7, 6, 5}};
    int g, b;
    for (g = 0; g < 3; ++g)
      for (b = 0; b < 6; ++b) {
        if (b == 4 && g == 2) continue; /* inflow: 1D/2D only */
        if (b == 5 && g != 1) continue; /* state sides: 2D only */
        for (s = 0; s < 3; ++s)
          for (h = 0; h < 4; ++h)
            grid_case(shapes[g][0], shapes[g][1], shapes[g][2], sets[b], s, h, h % 3);
      }
  }
  /* refusals */
  {
    double U[5 * 8], out[5 * 8], dt;
    orc_params_default(&p, 8, 1, 1, 0.1);
    expect(orc_rhs(NULL, 8, 1, 1, 0.1, 1.4, &p, out) < 0, "rhs refuses NULL");
    expect(orc_rhs(U, 0, 1, 1, 0.1, 1.4, &p, out) < 0, "rhs refuses an empty grid");
    expect(orc_rhs(U, 8, 1, 1, -0.1, 1.4, &p, out) < 0, "rhs refuses dx <= 0");
    expect(orc_cfl_dt(U, 8, 1, 1, 0.1, 1.4, 0.5, NULL) < 0, "cfl_dt refuses NULL");
    p.bc[0] = ORC_BC_INFLOW;
    p.inflow = NULL;
    expect(orc_rhs(U, 8, 1, 1, 0.1, 1.4, &p, out) < 0, "rhs refuses a missing inflow state");
    (void)dt;
  }
  if (failures) return 1;
  printf("oracle under sanitizers: ok\n");
  return 0;
}
