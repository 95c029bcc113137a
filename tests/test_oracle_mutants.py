"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a temporary copy of the oracle's C sources
(the files under oracle/ are not touched), builds it with the oracle's own
flags, and runs the CPU pin suites against that build in a child process
(ORACLE_L2IS_LIB).  Every planted mistake must make a pin fail.  The cases
are the kinds of slip the method invites: an index of the mirrored f-
stencil, a sign of the flux splitting, an L2 error term, a sign inside
tau5, the Roe density of the detector, a coefficient of the six-point
central flux, a Runge-Kutta weight, the mirror index of a reflective ghost,
weights of another WENO family (inverse-square smoothness weights), which
lose the fifth order on smooth data, and three readings the paper leaves
open: shear eigenvectors without the Roe sound speed, the LLF speed over
the face's two cells instead of its six-cell stencil, and a time step from
the fastest single direction instead of the sum over directions; and slips
in the comparison weightings, the moving boundary of the double Mach
reflection and the global LF speeds.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = ["tests/test_oracle_scalar.py", "tests/test_oracle_face.py", "tests/test_oracle_readings.py",
        "tests/test_oracle_solutions.py", "tests/test_oracle_dmr.py", "tests/test_oracle_inflow.py"]
# the jet's 1000-step robustness record is left out of the children (it pins
# no quantity of the definitions, and alone would take minutes on one thread)
PIN_FILTER = "not robustness"

# (name, file, text as written, planted mistake)
MUTANTS = [
    ("mirrored_stencil_offset", "face.c",
     "am[m] = fm[5 - m];", "am[m] = fm[4 - m];"),
    ("split_sign", "face.c",
     "fm[m] = 0.5 * (g[m] - alpha[s] * v[m]);", "fm[m] = 0.5 * (g[m] + alpha[s] * v[m]);"),
    ("E1_dropped", "weno_scalar.c",
     "E[1] = E[0];", "E[1] = 0.0;"),
    ("tau5_sign", "weno_scalar.c",
     "t2 = fp2 - 2.0 * fp1 + 2.0 * fm1 - fm2;", "t2 = fp2 - 2.0 * fp1 - 2.0 * fm1 - fm2;"),
    ("roe_density_arithmetic_mean", "charsys.c",
     "rhot = wl * wr;", "rhot = 0.5 * (pl[0] + pr[0]);"),
    ("central_flux_tap", "face.c",
     "37.0 * (F6[2][i] + F6[3][i])", "36.0 * (F6[2][i] + F6[3][i])"),
    ("rk_stage2_weights", "solver.c",
     "U2[k] = 0.75 * U[k] + 0.25 * (U1[k] + dt * Lk[k]);",
     "U2[k] = 0.25 * U[k] + 0.75 * (U1[k] + dt * Lk[k]);"),
    ("reflective_ghost_index", "solver.c",
     "return -1 - k;", "return -k;"),
    ("inverse_square_weights", "weno_scalar.c",
     "alpha[k] = d[k] * (1.0 + lam * tau5 / (lam * beta[k] + E[k] + eps_w));",
     "alpha[k] = d[k] / ((beta[k] + eps_w) * (beta[k] + eps_w));"),
    # shear eigenvectors without the Roe sound speed: the shear field's
    # characteristic variable then carries momentum units
    ("shear_eigenvectors_unscaled", "charsys.c",
     "    R[(1 + t) * nvar + s] = ct;\n"
     "    R[(nvar - 1) * nvar + s] = ct * ut[t];\n"
     "    L[s * nvar + 0] = -ut[t] / ct;\n"
     "    L[s * nvar + 1 + t] = 1.0 / ct;\n",
     "    R[(1 + t) * nvar + s] = 1.0;\n"
     "    R[(nvar - 1) * nvar + s] = ut[t];\n"
     "    L[s * nvar + 0] = -ut[t];\n"
     "    L[s * nvar + 1 + t] = 1.0;\n"),
    # LLF speed over the two cells of the face instead of the six-cell stencil
    ("llf_two_cells", "face.c",
     "for (m = 0; m < 6; ++m) {\n        double e = fabs(cell_eig(",
     "for (m = 2; m < 4; ++m) {\n        double e = fabs(cell_eig("),
    # the second term of beta_01 (Eq.(15)) with a wrong coefficient
    ("beta01_coefficient", "weno_scalar.c",
     "b01 = 13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2;",
     "b01 = 13.0 / 12.0 * t1 * t1 + 0.5 * t2 * t2;"),
    # the third RK stage evaluated at t + dt instead of t + dt/2 (a moving
    # state boundary sees it)
    ("stage3_time", "solver.c",
     "ps.time = p->time + 0.5 * dt;", "ps.time = p->time + dt;"),
    # the moving front's ghosts compared at the wrong height (the interior
    # row's centre instead of the ghost's)
    ("front_ghost_height", "solver.c",
     "yc = (k + 0.5) * g->dx;", "yc = (k - 0.5) * g->dx;"),
    # lambda of Eq.(32) from sqrt(sigma) instead of sigma
    ("lambda_sqrt_sigma", "face.c",
     "lr = p->c_reg * sig[s];", "lr = p->c_reg * sqrt(sig[s]);"),
    # the threshold of Eq.(35) with one power of dx/L too few
    ("threshold_power", "solver.c",
     "for (k = 0; k < p->thr_alpha; ++k) e *= r;", "for (k = 1; k < p->thr_alpha; ++k) e *= r;"),
    # the third RK stage's weights exchanged
    ("rk_stage3_weights", "solver.c",
     "U[k] = (1.0 / 3.0) * U[k] + (2.0 / 3.0) * (U2[k] + dt * Lk[k]);",
     "U[k] = (2.0 / 3.0) * U[k] + (1.0 / 3.0) * (U2[k] + dt * Lk[k]);"),
    # E_0 = E_1 of Eq.(27) with 1/36 instead of 1/45
    ("E01_constant", "weno_scalar.c",
     "E[0] = t1 * t1 / 45.0;", "E[0] = t1 * t1 / 36.0;"),
    # transmissive ghosts copying the second cell of the upper side
    ("transmissive_hi_index", "solver.c",
     "if (bchi == ORC_BC_TRANSMISSIVE) return n - 1;", "if (bchi == ORC_BC_TRANSMISSIVE) return n - 2;"),
    # periodic ghosts of the upper side shifted by one cell
    ("periodic_hi_index", "solver.c",
     "if (bchi == ORC_BC_PERIODIC) return k % n;", "if (bchi == ORC_BC_PERIODIC) return (k + 1) % n;"),
    # the time step blind to the speed of the inflow ghost states (Z24)
    ("cfl_without_inflow_speed", "solver.c",
     "      if (s > smax) smax = s;\n    }\n  }\n  *dt = p->cfl * dx / smax;",
     "      if (s > smax && 0) smax = s;\n    }\n  }\n  *dt = p->cfl * dx / smax;"),
    # Roe splitting speeds taken in the reverse field order
    ("roe_speed_field_order", "face.c",
     "alpha[s] = fabs(lam[s]);", "alpha[s] = fabs(lam[nvar - 1 - s]);"),
    # global LF speeds of the two acoustic fields exchanged
    ("lf_acoustic_fields_swapped", "solver.c",
     "double e = fabs(s == 0 ? un - cs : (s == g->nvar - 1 ? un + cs : un));",
     "double e = fabs(s == 0 ? un + cs : (s == g->nvar - 1 ? un - cs : un));"),
    # time step from the largest single-direction speed instead of the sum
    ("cfl_max_over_directions", "solver.c",
     "for (d = 0; d < g->dim; ++d) s += fabs(prim[1 + d]) + prim[5];\n    if (s > smax || s != s)",
     "for (d = 0; d < g->dim; ++d) s = fmax(s, fabs(prim[1 + d]) + prim[5]);\n    if (s > smax || s != s)"),
]


# the unaltered sources through the same copy / build / load route: the pins
# must pass, so a failure of a mutant is the planted mistake's doing
CONTROL = ("control_unaltered", "face.c", "am[m] = fm[5 - m];", "am[m] = fm[5 - m];")


def test_planted_mistakes_fail_a_pin(tmp_path):
    from oracle import pyoracle
    procs = []
    for name, fname, old, new in [CONTROL] + MUTANTS:
        d = tmp_path / name
        d.mkdir()
        for f in os.listdir(ORACLE):
            if f.endswith((".c", ".h")):
                shutil.copy(os.path.join(ORACLE, f), d / f)
        src = (d / fname).read_text()
        assert src.count(old) == 1, (name, "text not found once in " + fname)
        (d / fname).write_text(src.replace(old, new))
        lib = str(d / "liboracle_mutant.so")
        pyoracle.build(src_dir=str(d), out=lib)
        env = dict(os.environ, ORACLE_L2IS_LIB=lib, OMP_NUM_THREADS="1")
        cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
               "-m", "not gpu", "-k", PIN_FILTER, *PINS]
        procs.append((name, subprocess.Popen(cmd, cwd=ROOT, env=env, stdout=subprocess.PIPE,
                                             stderr=subprocess.STDOUT, text=True)))
    survived = []
    for name, p in procs:
        out, _ = p.communicate(timeout=600)
        if name == CONTROL[0]:
            assert p.returncode == 0, out[-2000:]
            continue
        # exit code 1: tests ran and at least one failed
        if p.returncode != 1 or "FAILED" not in out:
            survived.append((name, p.returncode, out.strip().splitlines()[-1:]))
    assert not survived, survived
