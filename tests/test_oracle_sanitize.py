"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and driven through operators, Jacobi-PCG, the GKB
solve and the saddle residual on small 2D and 3D grids: any out-of-bounds
access, leak or undefined operation fails the run."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
typedef struct { int dim; int n[3]; double h; int bc[6]; int pin; } og_grid;
typedef struct {
  double tol; int delay; int maxit; double inner_tol; int inner_maxit; int squared_rule;
  double *zeta, *alpha, *beta, *est_hist; int *inner_iters; int store_k; double *V, *Q;
  int inner_krylov; int restart;
} og_gkb_opts;
long og_m_full(const og_grid *g);
long og_n_cells(const og_grid *g);
int og_gkb_solve(const og_grid *g, const double *mu, double eta, const double *gv,
                 const double *rv, const og_gkb_opts *o, double *w, double *p,
                 int *K_out, double *est_out, int *inner_total);
void og_saddle_residual(const og_grid *g, const double *mu, const double *gv,
                        const double *rv, const double *w, const double *p,
                        double *res_w, double *res_r, double *norms);
int og_gkb_fgmres(const og_grid *g, const double *mu, double eta, const double *gv,
                  const double *rv, const og_gkb_opts *o, double tol, int restart, int maxit,
                  double *w, double *p, int *iters, int *inner_total);

static int run(og_grid g, int varmu, double eta) {
  long mf = og_m_full(&g), nc = og_n_cells(&g);
  double *gv = malloc(mf * sizeof(double)), *w = malloc(mf * sizeof(double));
  double *rv = calloc(nc, sizeof(double)), *p = malloc(nc * sizeof(double));
  double *mu = varmu ? malloc(nc * sizeof(double)) : NULL;
  double *zeta = malloc(300 * sizeof(double)), *est = malloc(300 * sizeof(double));
  int *inner = malloc(301 * sizeof(int));
  for (long i = 0; i < mf; ++i) gv[i] = sin(0.37 * (double)i) + 0.1;
  for (long i = 0; i < nc && mu; ++i) mu[i] = 1.0 + (double)(i % 3);
  og_gkb_opts o = {1e-10, 3, 300, 1e-13, 100000, 0, zeta, NULL, NULL, est, inner, 0, NULL, NULL};
  int K = 0, tot = 0;
  double e = 0.0, norms[4];
  int st = og_gkb_solve(&g, mu, eta, gv, rv, &o, w, p, &K, &e, &tot);
  double *resw = malloc(mf * sizeof(double)), *resr = malloc(nc * sizeof(double));
  og_saddle_residual(&g, mu, gv, rv, w, p, resw, resr, norms);
  printf("dim %d status %d K %d inner %d residual %.3e\n", g.dim, st, K, tot, norms[0] / norms[3]);
  int ok = st == 0 && norms[0] <= 1e-7 * norms[3];
  /* FGMRES inner solves (restart 7) and GKB as the preconditioner of an
     outer FGMRES (restart 3) on the same system */
  o.inner_krylov = 1;
  o.restart = 7;
  st = og_gkb_solve(&g, mu, eta, gv, rv, &o, w, p, &K, &e, &tot);
  og_saddle_residual(&g, mu, gv, rv, w, p, resw, resr, norms);
  ok = ok && st == 0 && norms[0] <= 1e-7 * norms[3];
  o.tol = 1e-2;
  o.delay = 2;
  int its = 0;
  st = og_gkb_fgmres(&g, mu, eta, gv, rv, &o, 1e-9, 3, 40, w, p, &its, &tot);
  og_saddle_residual(&g, mu, gv, rv, w, p, resw, resr, norms);
  printf("  fgmres inner / gkb-preconditioned fgmres: status %d its %d residual %.3e\n", st, its,
         norms[0] / norms[3]);
  ok = ok && st == 0 && norms[0] <= 1e-8 * norms[3];
  free(resw); free(resr);
  free(gv); free(w); free(rv); free(p); free(mu); free(zeta); free(est); free(inner);
  return ok ? 0 : 1;
}

int main(void) {
  og_grid a = {2, {12, 6, 1}, 1.0 / 6.0, {0, 1, 0, 0, 0, 0}, -1};  /* natural outflow */
  og_grid b = {3, {6, 4, 5}, 0.25, {0, 0, 0, 0, 0, 0}, 0};          /* box, pinned cell */
  og_grid c = {3, {4, 6, 4}, 0.25, {1, 0, 0, 0, 0, 0}, -1};         /* natural lower side */
  return run(a, 0, 10.0) | run(b, 1, 100.0) | run(c, 1, 0.0);
}
"""


def _sanitizers_available(tmp):
    probe = os.path.join(tmp, "probe.c")
    with open(probe, "w") as f:
        f.write("int main(void){return 0;}\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", "-o", os.path.join(tmp, "probe"),
                        probe], capture_output=True)
    return r.returncode == 0


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    tmp = str(tmp_path)
    if not _sanitizers_available(tmp):
        pytest.skip("gcc sanitizer runtime not available")
    drv = os.path.join(tmp, "driver.c")
    with open(drv, "w") as f:
        f.write(DRIVER)
    exe = os.path.join(tmp, "driver")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
                    drv, SRC, "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    if r.returncode != 0 and "LeakSanitizer does not work" in r.stderr:
        env["ASAN_OPTIONS"] = "detect_leaks=0"
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert r.stdout.count("status 0") == 6  # three GKB solves, three FGMRES runs
