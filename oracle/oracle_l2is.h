/*
 * CPU oracle for the L2-norm regularized incremental-stencil WENO scheme
 * (Zhu & Hu, "A L2-norm regularized incremental-stencil WENO scheme for
 * compressible flows", arXiv 1908.02464) applied to the compressible Euler
 * equations on uniform 1D/2D/3D grids.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, scalar FP64 reference
 * written from the paper.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no source with the
 * GPU library and must never be used as a fallback for it.
 *
 * Layout of every state array: structure of arrays [nvar][nz][ny][nx],
 * x fastest, interior cells only.  nvar = 2 + dim, with
 * dim = 1 (ny == nz == 1), 2 (nz == 1, ny > 1) or 3 (nz > 1, ny > 1).
 * Variables: rho, rho*u_x, [rho*u_y, [rho*u_z]], E.
 *
 * Return codes: 0 ok, < 0 invalid argument, 1 non-physical state found.
 *
 * Pins (CPU tests, against what the paper and the mathematics fix): the
 * reconstruction and its weightings against the integral definitions of
 * Eq.(9), (10), (26) and their limits; the eigensystem against L R = I and
 * the complex-step Jacobian; the face flux against the optimal-weight
 * identity of Eq.(34) and the readings of the open points; the right-hand
 * side and the steps against conservation, symmetries, changes of units,
 * exact Riemann solutions (Toro's star states), convergence orders and
 * grids extended by their ghost cells; dt against its definition.  Parity
 * unpinned for whole-scheme values at the paper's own workloads: the paper
 * prints no number of the scheme's output to compare with (its figures
 * are missing from the available text), so those runs rest on the pins
 * above.
 */
#ifndef ORACLE_L2IS_H
#define ORACLE_L2IS_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_TRANSMISSIVE = 1, ORC_BC_REFLECTIVE = 2,
       ORC_BC_INFLOW = 3,      /* x- side of a 1D/2D grid: ghosts = inflow[]  */
       ORC_BC_STATE_WALL = 4,  /* y side of a 2D grid: ghosts of the cells with
                                  centre x < bgeom[0] hold bstate[0], the
                                  others mirror the interior (a wall)          */
       ORC_BC_STATE_FRONT = 5  /* y side of a 2D grid: a ghost centred at
                                  (x, y) holds bstate[0] if x < bgeom[1] +
                                  bgeom[2] y + bgeom[3] time, else bstate[1]
                                  (a straight front moving along x)           */
};
enum { ORC_SPLIT_LLF = 0, ORC_SPLIT_LF = 1, ORC_SPLIT_ROE = 2 };
enum {
  ORC_HYB_PER_FIELD = 0,  /* linear flux for field s iff sigma^s < eps      */
  ORC_HYB_PER_FACE = 1,   /* linear for all fields iff max_s sigma^s < eps  */
  ORC_HYB_WENO_ONLY = 2,  /* never linear (pure regularized WENO-IS)        */
  ORC_HYB_LINEAR_ONLY = 3 /* always linear (optimal upwind scheme)          */
};

enum {
  ORC_W_L2IS = 0,   /* regularized weights of the present scheme, Eq.(28)    */
  ORC_W_IS = 1,     /* original WENO-IS weights, Eq.(8)                       */
  ORC_W_IS_B01 = 2  /* WENO-IS with beta_01 on the 2-point stencils,
                       Eq.(14)-(15) (the "WENO-IS" of the comparisons)       */
};

typedef struct {
  double cfl;       /* CFL number (Sec. 4: 0.5)                                */
  double c_reg;     /* c in lambda = c * sigma, Eq.(32): 1                     */
  double eps_w;     /* epsilon in the weights, Eq.(8)/(28): 1e-20              */
  double thr_C;     /* C in the threshold eps = C (dx/L)^alpha, Eq.(35): 1     */
  int thr_alpha;    /* alpha in Eq.(35): 3                                     */
  int split;        /* ORC_SPLIT_*                                             */
  int hybrid;       /* ORC_HYB_*                                               */
  int bc[6];        /* x-, x+, y-, y+, z-, z+ : ORC_BC_*                       */
  double thr_L[3];  /* characteristic length L per direction in Eq.(35)       */
  const double *inflow; /* ORC_BC_INFLOW on bc[0]: the conserved state of the
                           ghosts left of x line y, inflow[v*ny + y]; else
                           unused (Sec. 4.7, the jet's left boundary)      */
  int weights;      /* ORC_W_*: weights of the nonlinear reconstruction       */
  double bstate[2][5];  /* conserved states of the STATE_WALL / STATE_FRONT
                           ghosts (first nvar values of each)                 */
  double bgeom[4];  /* x of the wall's start; x0, dx/dy, dx/dt of the front   */
  double time;      /* time of the state (stage time inside orc_step; the
                       start time of orc_run); read by STATE_FRONT            */
} orc_params;

/* Fill defaults for a grid: thr_L[d] = n_d * dx, transmissive boundaries,
 * inflow = NULL, weights ORC_W_L2IS, boundary states and geometry zero,
 * time 0.  Cell centres lie at ((i + 1/2) dx, (j + 1/2) dx, ...). */
int orc_params_default(orc_params *p, int nx, int ny, int nz, double dx);

/* Scalar WENO-L2IS reconstruction at x_{j+1/2} from a[0..4] = f_{j-2..j+2}
 * with regularization parameter lam (Eq.(5),(6),(11),(27),(28)).
 * dbg (may be NULL) receives 17 values:
 *   q0..q3, beta0..beta3, tau5, E0..E3, omega0..omega3. */
double orc_weno_l2is(const double a[5], double lam, double eps_w, double *dbg);

/* The same reconstruction with the weights `weights` (ORC_W_*); lam is read
 * by ORC_W_L2IS only.  dbg as above (E_k is computed in every case). */
double orc_weno(const double a[5], int weights, double lam, double eps_w, double *dbg);

/* Roe average between UL and UR and the eigensystem of the Roe Jacobian along
 * direction dir (0,1,2).  L and R are nvar x nvar row-major, L = R^{-1};
 * column s of R is the right eigenvector of field s, row s of L the left one.
 * Field order: u_n - c, u_n (entropy), shear fields (tangential momentum in
 * increasing index order), u_n + c.  lam: eigenvalues per field.
 * roe (may be NULL): rho~, u~_x, u~_y, u~_z, H~, c~ (6 values). */
int orc_roe_eigen(int nvar, int dir, double gamma, const double *UL,
                  const double *UR, double *L, double *R, double *lam,
                  double *roe);

/* Physical flux along dir of one state, and its primitive variables.
 * prim (may be NULL): rho, u_x, u_y, u_z, p, c, H (7 values). */
int orc_phys_flux(int nvar, int dir, double gamma, const double *U, double *F,
                  double *prim);

/* Numerical flux at one face x_{j+1/2} from the six states U6[m*nvar + i],
 * m = 0..5 meaning cells j-2..j+3 (already with boundary ghosts applied).
 * eps_thr is the switch threshold for this direction; alpha_lf (length nvar)
 * is only read for ORC_SPLIT_LF.  flags[s] = 1 if field s took the linear flux;
 * sigma[s] = detector value of Eq.(30).  flags/sigma may be NULL. */
int orc_face_flux(int nvar, int dir, double gamma, const orc_params *p,
                  double eps_thr, const double *alpha_lf, const double *U6,
                  double *Fhat, unsigned char *flags, double *sigma);

/* dU/dt of Eq.(19), summed over the active directions. */
int orc_rhs(const double *U, int nx, int ny, int nz, double dx, double gamma,
            const orc_params *p, double *dUdt);

/* dU/dt at ncells selected cells only; cell[k] = x + nx*(y + ny*z).
 * out[v*ncells + k].  For ORC_SPLIT_LF the global speeds are taken over the
 * whole grid. */
int orc_rhs_at(const double *U, int nx, int ny, int nz, double dx,
               double gamma, const orc_params *p, int ncells,
               const long long *cell, double *out);

/* Per-face flags and detector values along dir for the whole grid.
 * Layout [nvar][..] with n_dir + 1 faces along dir (face f between cells f-1
 * and f), the other two extents unchanged, x fastest. */
int orc_face_debug(const double *U, int nx, int ny, int nz, double dx,
                   double gamma, const orc_params *p, int dir,
                   unsigned char *flags, double *sigma);

/* CFL time step dt = cfl * dx / max_cells sum_d (|u_d| + c).
 * Returns 1 (and still writes dt) if some cell is non-physical. */
int orc_cfl_dt(const double *U, int nx, int ny, int nz, double dx,
               double gamma, double cfl, double *dt);

/* One third-order SSP Runge-Kutta step in place from time p->time.  dt_in >
 * 0: use it; otherwise the CFL dt of the current state, whose maximum speed
 * also takes the inflow ghost states of an ORC_BC_INFLOW side.  The stages
 * evaluate the right-hand side at times t, t + dt, t + dt/2 (the times of
 * the Shu-Osher stages).  dt_used may be NULL. */
int orc_step(double *U, int nx, int ny, int nz, double dx, double gamma,
             const orc_params *p, double dt_in, double *dt_used);

/* Threads used for the lines of a direction (built with OpenMP; else 1).
 * n > 0 sets the count; returns the count in effect.  Results do not depend
 * on it. */
int orc_threads(int n);

/* Advance from p->time to t_end (last step clipped) or max_steps, whichever
 * first.
 * Returns the status of the last check. */
int orc_run(double *U, int nx, int ny, int nz, double dx, double gamma,
            const orc_params *p, double t_end, int max_steps, double *t_out,
            int *steps_out);

#ifdef __cplusplus
}
#endif
#endif
