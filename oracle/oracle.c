/*
 * CPU FP64 oracle for the generalized Golub-Kahan bidiagonalization (GKB)
 * solver of the saddle-point system [[W, A], [A^T, 0]] [w; p] = [g; r]
 * on a MAC (staggered) grid.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library: operators, inner solver, GKB recurrence and stopping
 * rule are all written out here, plainly, in double precision.
 *
 * What it follows:
 *   - augmented matrix M = W + gamma A N^-1 A^T with N = (1/eta) I, gamma = 1
 *     for eta > 0 and gamma = 0, N = I for eta = 0 (paper Section 2, eq. for
 *     M, and the option table of Section 3);
 *   - the transformation to a zero first right-hand side (Section 2, the
 *     change of variables u = w - M^-1(g + gamma A N^-1 r),
 *     b = r - A^T M^-1(g + gamma A N^-1 r));
 *   - the Craig-variant GKB recurrence (Section 2.1, Algorithm 1);
 *   - the delayed lower-bound stopping rule (Section 2.2), read with the
 *     non-squared ratio: stop when sqrt(sum of the newest d+1 zeta_j^2 /
 *     sum of all zeta_j^2) <= tau;
 *   - the inner solve with M by Jacobi-preconditioned CG started from 0,
 *     stopped on the relative unpreconditioned residual (Section 4.1.3).
 *
 * Discretization (MAC, strong-form scaling): W is the component-wise
 * viscous operator -div(mu grad u_c); normal-direction couplings use the
 * cell viscosity between the two faces, tangential couplings the arithmetic
 * mean of the cells that touch the edge between them.  DIRICHLET walls:
 * faces normal to the wall are not unknowns (value 0 in the homogeneous
 * operator); tangential wall ghosts are mirrored (ghost = -u_f).  NATURAL
 * (do-nothing) sides: normal faces are unknowns owning half a control volume
 * (tangential terms halved), couplings across the side are absent.
 * A is the gradient (p_R - p_L)/h with missing or pinned cells read as 0;
 * A^T is its exact transpose.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OG_DIRICHLET 0
#define OG_NATURAL 1

#define OG_OK 0
#define OG_MAXIT 1
#define OG_EINVAL -1
#define OG_ENOMEM -2
#define OG_ENAN -4
#define OG_EINNER -5

typedef struct {
  int dim;
  int n[3];
  double h;
  int bc[6];
  int pin;
} og_grid;

/* ------------------------------------------------------------------ layout */

static long og_nz(const og_grid *g) { return g->dim == 3 ? g->n[2] : 1; }

/* extents (x, y, z) of the face array of component c */
static void comp_ext(const og_grid *g, int c, long e[3]) {
  e[0] = g->n[0];
  e[1] = g->n[1];
  e[2] = og_nz(g);
  e[c] += 1;
}

static long comp_size(const og_grid *g, int c) {
  long e[3];
  comp_ext(g, c, e);
  return e[0] * e[1] * e[2];
}

static long comp_off(const og_grid *g, int c) {
  long o = 0;
  for (int a = 0; a < c; ++a) o += comp_size(g, a);
  return o;
}

long og_m_full(const og_grid *g) {
  long m = 0;
  for (int c = 0; c < g->dim; ++c) m += comp_size(g, c);
  return m;
}

long og_n_cells(const og_grid *g) { return (long)g->n[0] * g->n[1] * og_nz(g); }

static long face_index(const og_grid *g, int c, const long P[3]) {
  long e[3];
  comp_ext(g, c, e);
  return comp_off(g, c) + (P[2] * e[1] + P[1]) * e[0] + P[0];
}

static long cell_index(const og_grid *g, const long P[3]) {
  return (P[2] * g->n[1] + P[1]) * (long)g->n[0] + P[0];
}

static int cell_exists(const og_grid *g, const long P[3]) {
  for (int a = 0; a < g->dim; ++a)
    if (P[a] < 0 || P[a] >= g->n[a]) return 0;
  return 1;
}

/* a face of component c at normal index ic is an unknown unless it lies on a
   DIRICHLET side */
static int face_unknown(const og_grid *g, int c, long ic) {
  if (ic == 0) return g->bc[2 * c] == OG_NATURAL;
  if (ic == g->n[c]) return g->bc[2 * c + 1] == OG_NATURAL;
  return 1;
}

static double mu_cell(const og_grid *g, const double *mu, const long P[3]) {
  return mu ? mu[cell_index(g, P)] : 1.0;
}

/* viscosity on the edge between face (c, P) and its neighbour along axis a
   (a != c) in direction s: arithmetic mean over the existing cells touching
   the edge (cells P[c]-1, P[c] along c; e-1, e along a; P[b] along b) */
static double mu_edge(const og_grid *g, const double *mu, int c, int a, int s,
                      const long P[3]) {
  long e = P[a] + (s > 0 ? 1 : 0);
  double sum = 0.0;
  int cnt = 0;
  for (int dc = -1; dc <= 0; ++dc)
    for (int da = -1; da <= 0; ++da) {
      long Q[3] = {P[0], P[1], P[2]};
      Q[c] = P[c] + dc;
      Q[a] = e + da;
      if (!cell_exists(g, Q)) continue;
      sum += mu_cell(g, mu, Q);
      ++cnt;
    }
  return sum / cnt;
}

/* decode a flat face index into (component, position) */
static void face_decode(const og_grid *g, long f, int *c, long P[3]) {
  int cc = 0;
  while (cc + 1 < g->dim && f >= comp_off(g, cc + 1)) ++cc;
  long e[3];
  comp_ext(g, cc, e);
  long l = f - comp_off(g, cc);
  P[0] = l % e[0];
  P[1] = (l / e[0]) % e[1];
  P[2] = l / (e[0] * e[1]);
  *c = cc;
}

/* --------------------------------------------------------------- operators */

/* (W x)_f for the unknown face (c, P); x_f is read from x; neighbours that
   are DIRICHLET faces read as 0 unless `ext` (then their stored value is used,
   and tangential wall ghosts use 2*wall - x_f with wall from wall_tan) */
static double W_row(const og_grid *g, const double *mu, const double *x, int c,
                    const long P[3], int ext, const double *wall_tan) {
  double xf = x[face_index(g, c, P)];
  double acc = 0.0;
  for (int a = 0; a < g->dim; ++a) {
    if (a == c) {
      for (int s = -1; s <= 1; s += 2) {
        long Q[3] = {P[0], P[1], P[2]};
        Q[c] += s;
        if (Q[c] < 0 || Q[c] > g->n[c]) continue; /* beyond a NATURAL side */
        long C[3] = {P[0], P[1], P[2]};
        C[c] = P[c] + (s < 0 ? -1 : 0);
        double kap = mu_cell(g, mu, C);
        double xn = (face_unknown(g, c, Q[c]) || ext) ? x[face_index(g, c, Q)] : 0.0;
        acc += kap * (xf - xn);
      }
    } else {
      double wgt = (P[c] == 0 || P[c] == g->n[c]) ? 0.5 : 1.0;
      for (int s = -1; s <= 1; s += 2) {
        long Q[3] = {P[0], P[1], P[2]};
        Q[a] += s;
        double kap = mu_edge(g, mu, c, a, s, P);
        if (Q[a] < 0 || Q[a] >= g->n[a]) {
          int side = 2 * a + (s > 0 ? 1 : 0);
          if (g->bc[side] == OG_DIRICHLET) {
            double wall = (ext && wall_tan) ? wall_tan[side * 3 + c] : 0.0;
            acc += wgt * kap * (xf - (2.0 * wall - xf));
          }
        } else {
          acc += wgt * kap * (xf - x[face_index(g, c, Q)]);
        }
      }
    }
  }
  return acc / (g->h * g->h);
}

static void apply_W_impl(const og_grid *g, const double *mu, const double *x,
                         double *y, int ext, const double *wall_tan) {
  long mf = og_m_full(g);
#pragma omp parallel for schedule(static)
  for (long f = 0; f < mf; ++f) {
    int c;
    long P[3];
    face_decode(g, f, &c, P);
    y[f] = face_unknown(g, c, P[c]) ? W_row(g, mu, x, c, P, ext, wall_tan) : 0.0;
  }
}

void og_apply_W(const og_grid *g, const double *mu, const double *x, double *y) {
  apply_W_impl(g, mu, x, y, 0, NULL);
}

/* W applied to a field that carries Dirichlet data: values stored at faces
   normal to DIRICHLET sides are used, tangential walls move with
   wall_tan[side*3 + component] (NULL = at rest).  Rows of unknown faces only. */
void og_apply_W_ext(const og_grid *g, const double *mu, const double *x,
                    const double *wall_tan, double *y) {
  apply_W_impl(g, mu, x, y, 1, wall_tan);
}

void og_apply_A(const og_grid *g, const double *p, double *y) {
  long mf = og_m_full(g);
#pragma omp parallel for schedule(static)
  for (long f = 0; f < mf; ++f) {
    int c;
    long P[3];
    face_decode(g, f, &c, P);
    if (!face_unknown(g, c, P[c])) {
      y[f] = 0.0;
      continue;
    }
    long R[3] = {P[0], P[1], P[2]}, L[3] = {P[0], P[1], P[2]};
    L[c] -= 1;
    double pr = 0.0, pl = 0.0;
    if (cell_exists(g, R) && cell_index(g, R) != g->pin) pr = p[cell_index(g, R)];
    if (cell_exists(g, L) && cell_index(g, L) != g->pin) pl = p[cell_index(g, L)];
    y[f] = (pr - pl) / g->h;
  }
}

void og_apply_AT(const og_grid *g, const double *x, double *t) {
  long nc = og_n_cells(g);
#pragma omp parallel for schedule(static)
  for (long q = 0; q < nc; ++q) {
    long P[3] = {q % g->n[0], (q / g->n[0]) % g->n[1], q / ((long)g->n[0] * g->n[1])};
    if (q == g->pin) {
      t[q] = 0.0;
      continue;
    }
    double acc = 0.0;
    for (int c = 0; c < g->dim; ++c) {
      long lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
      hi[c] += 1;
      if (face_unknown(g, c, lo[c])) acc += x[face_index(g, c, lo)];
      if (face_unknown(g, c, hi[c])) acc -= x[face_index(g, c, hi)];
    }
    t[q] = acc / g->h;
  }
}

/* y = W x + eta A (A^T x); eta = 0 gives y = W x */
void og_apply_M(const og_grid *g, const double *mu, double eta, const double *x,
                double *y) {
  long mf = og_m_full(g), nc = og_n_cells(g);
  og_apply_W(g, mu, x, y);
  if (eta == 0.0) return;
  double *t = malloc(sizeof(double) * nc);
  double *z = malloc(sizeof(double) * mf);
  og_apply_AT(g, x, t);
  og_apply_A(g, t, z);
  for (long f = 0; f < mf; ++f) y[f] += eta * z[f];
  free(t);
  free(z);
}

/* diagonal of M (0 at non-unknown faces) */
void og_diag_M(const og_grid *g, const double *mu, double eta, double *d) {
  long mf = og_m_full(g);
  double h2 = g->h * g->h;
#pragma omp parallel for schedule(static)
  for (long f = 0; f < mf; ++f) {
    int c;
    long P[3];
    face_decode(g, f, &c, P);
    if (!face_unknown(g, c, P[c])) {
      d[f] = 0.0;
      continue;
    }
    double acc = 0.0;
    for (int a = 0; a < g->dim; ++a) {
      if (a == c) {
        for (int s = -1; s <= 1; s += 2) {
          long Q[3] = {P[0], P[1], P[2]};
          Q[c] += s;
          if (Q[c] < 0 || Q[c] > g->n[c]) continue;
          long C[3] = {P[0], P[1], P[2]};
          C[c] = P[c] + (s < 0 ? -1 : 0);
          acc += mu_cell(g, mu, C);
        }
      } else {
        double wgt = (P[c] == 0 || P[c] == g->n[c]) ? 0.5 : 1.0;
        for (int s = -1; s <= 1; s += 2) {
          long Q[3] = {P[0], P[1], P[2]};
          Q[a] += s;
          double kap = mu_edge(g, mu, c, a, s, P);
          if (Q[a] < 0 || Q[a] >= g->n[a]) {
            if (g->bc[2 * a + (s > 0 ? 1 : 0)] == OG_DIRICHLET) acc += wgt * 2.0 * kap;
          } else {
            acc += wgt * kap;
          }
        }
      }
    }
    double dd = acc / h2;
    if (eta != 0.0) {
      long R[3] = {P[0], P[1], P[2]}, L[3] = {P[0], P[1], P[2]};
      L[c] -= 1;
      int cnt = 0;
      if (cell_exists(g, R) && cell_index(g, R) != g->pin) ++cnt;
      if (cell_exists(g, L) && cell_index(g, L) != g->pin) ++cnt;
      dd += eta * cnt / h2;
    }
    d[f] = dd;
  }
}

/* ------------------------------------------------------------ vector utils */

static double dot(long n, const double *a, const double *b) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

static int all_zero(long n, const double *a) {
  for (long i = 0; i < n; ++i)
    if (a[i] != 0.0) return 0;
  return 1;
}

/* ------------------------------------------------------ Jacobi-PCG on M */

/* Solve M x = f by CG with the Jacobi preconditioner diag(M)^-1, x0 = 0.
   Stops when ||f - M x_i||_2 <= tol ||f||_2 (recursive residual) or after
   maxit iterations.  Returns OG_OK or OG_EINNER; *iters = iterations done. */
int og_pcg(const og_grid *g, const double *mu, double eta, const double *f,
           double *x, double tol, int maxit, int *iters) {
  long mf = og_m_full(g);
  double *r = malloc(sizeof(double) * mf), *z = malloc(sizeof(double) * mf);
  double *p = malloc(sizeof(double) * mf), *q = malloc(sizeof(double) * mf);
  double *dg = malloc(sizeof(double) * mf);
  if (!r || !z || !p || !q || !dg) return OG_ENOMEM;
  og_diag_M(g, mu, eta, dg);
  for (long i = 0; i < mf; ++i) {
    x[i] = 0.0;
    r[i] = f[i];
    z[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0;
    p[i] = z[i];
  }
  double rr0 = dot(mf, f, f);
  double rz = dot(mf, r, z);
  int it = 0, status = OG_EINNER;
  if (rr0 == 0.0) status = OG_OK;
  while (status != OG_OK && it < maxit) {
    og_apply_M(g, mu, eta, p, q);
    double pq = dot(mf, p, q);
    double alpha = rz / pq;
    for (long i = 0; i < mf; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    ++it;
    double rr = dot(mf, r, r);
    if (!isfinite(rr)) {
      status = OG_ENAN;
      break;
    }
    if (rr <= tol * tol * rr0) {
      status = OG_OK;
      break;
    }
    for (long i = 0; i < mf; ++i) z[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0;
    double rz_new = dot(mf, r, z);
    double beta = rz_new / rz;
    rz = rz_new;
    for (long i = 0; i < mf; ++i) p[i] = z[i] + beta * p[i];
  }
  if (iters) *iters = it;
  free(r);
  free(z);
  free(p);
  free(q);
  free(dg);
  return status;
}

/* ---------------------------------------------------------------- GKB */

typedef struct {
  double tol;         /* tau of the lower-bound rule; <= 0 runs to maxit */
  int delay;          /* d */
  int maxit;          /* maximum number of zeta values (K) */
  double inner_tol;   /* relative residual of each inner Jacobi-PCG solve */
  int inner_maxit;
  int squared_rule;   /* 1: literal squared comparison xi^2 <= tau * sum */
  /* optional outputs */
  double *zeta;       /* [maxit] zeta_1..zeta_K */
  double *alpha;      /* [maxit] alpha_1..alpha_K */
  double *beta;       /* [maxit] beta_1..beta_K (beta_1 = ||b||_{N^-1}) */
  double *est_hist;   /* [maxit] lower-bound ratio after each K (>= d+1), else -1 */
  int *inner_iters;   /* [maxit + 1] inner iterations of each M-solve */
  int store_k;        /* number of V and Q columns to store */
  double *V;          /* [store_k][m_full] */
  double *Q;          /* [store_k][n_cells] */
} og_gkb_opts;

/* Solve [[W, A], [A^T, 0]] [w; p] = [g; r].  Returns OG_OK, OG_MAXIT or an
   error; *K = number of zeta values computed, *est = last lower-bound ratio. */
int og_gkb_solve(const og_grid *g, const double *mu, double eta, const double *gv,
                 const double *rv, const og_gkb_opts *o, double *w, double *p,
                 int *K_out, double *est_out, int *inner_total) {
  long mf = og_m_full(g), nc = og_n_cells(g);
  if (eta < 0.0 || o->delay < 0 || o->maxit < 1) return OG_EINVAL;
  double ninv = eta > 0.0 ? eta : 1.0; /* N^-1 = ninv * I */
  double *ghat = calloc(mf, sizeof(double)), *w0 = calloc(mf, sizeof(double));
  double *u = calloc(mf, sizeof(double)), *v = calloc(mf, sizeof(double));
  double *Mv = calloc(mf, sizeof(double)), *s = calloc(mf, sizeof(double));
  double *y = calloc(mf, sizeof(double)), *f = calloc(mf, sizeof(double));
  double *b = calloc(nc, sizeof(double)), *q = calloc(nc, sizeof(double));
  double *d = calloc(nc, sizeof(double)), *t = calloc(nc, sizeof(double));
  double *mask = calloc(mf, sizeof(double));
  int status = OG_OK, K = 0, its = 0, tot = 0, solve_idx = 0;
  double est = 1.0;

  double *zs = calloc(o->maxit + 1, sizeof(double)); /* zeta_1 .. zeta_K */
  /* unknown-face mask: the diagonal of W is positive exactly there */
  og_diag_M(g, mu, 0.0, mask);
  for (long i = 0; i < mf; ++i) mask[i] = mask[i] > 0.0 ? 1.0 : 0.0;

  /* transformation: ghat = g + gamma A N^-1 r, w0 = M^-1 ghat, b = r - A^T w0 */
  for (long i = 0; i < mf; ++i) ghat[i] = gv[i] * mask[i];
  if (eta > 0.0) {
    double *rr = malloc(sizeof(double) * nc), *Ar = malloc(sizeof(double) * mf);
    for (long i = 0; i < nc; ++i) rr[i] = (i == g->pin) ? 0.0 : rv[i];
    og_apply_A(g, rr, Ar);
    for (long i = 0; i < mf; ++i) ghat[i] += eta * Ar[i];
    free(rr);
    free(Ar);
  }
  if (!all_zero(mf, ghat)) {
    int st = og_pcg(g, mu, eta, ghat, w0, o->inner_tol, o->inner_maxit, &its);
    tot += its;
    if (o->inner_iters) o->inner_iters[solve_idx] = its;
    if (st != OG_OK) { status = st; goto done; }
  }
  ++solve_idx;
  og_apply_AT(g, w0, b);
  for (long i = 0; i < nc; ++i) b[i] = ((i == g->pin) ? 0.0 : rv[i]) - b[i];

  /* initialisation of Algorithm 1 */
  double beta1 = sqrt(ninv * dot(nc, b, b));
  for (long i = 0; i < nc; ++i) p[i] = 0.0;
  if (beta1 == 0.0) {
    est = 0.0;
    goto finish;
  }
  for (long i = 0; i < nc; ++i) q[i] = ninv * b[i] / beta1;
  og_apply_A(g, q, f);
  {
    int st = og_pcg(g, mu, eta, f, s, o->inner_tol, o->inner_maxit, &its);
    tot += its;
    if (o->inner_iters) o->inner_iters[solve_idx] = its;
    ++solve_idx;
    if (st != OG_OK) { status = st; goto done; }
  }
  og_apply_M(g, mu, eta, s, y);
  double alpha = sqrt(dot(mf, s, y));
  if (!isfinite(alpha) || alpha == 0.0) { status = OG_ENAN; goto done; }
  for (long i = 0; i < mf; ++i) {
    v[i] = s[i] / alpha;
    Mv[i] = y[i] / alpha;
  }
  double zeta = beta1 / alpha;
  for (long i = 0; i < nc; ++i) {
    d[i] = q[i] / alpha;
    p[i] = -zeta * d[i];
  }
  for (long i = 0; i < mf; ++i) u[i] = zeta * v[i];
  K = 1;
  double sum_all = zeta * zeta;
  zs[0] = zeta;
  if (o->zeta) o->zeta[0] = zeta;
  if (o->alpha) o->alpha[0] = alpha;
  if (o->beta) o->beta[0] = beta1;
  if (o->est_hist) o->est_hist[0] = -1.0;
  if (o->store_k > 0) {
    memcpy(o->V, v, sizeof(double) * mf);
    memcpy(o->Q, q, sizeof(double) * nc);
  }

  int converged = 0;
  while (!converged && K < o->maxit) {
    /* t = N^-1 (A^T v_k - alpha_k N q_k), beta = ||t||_N */
    og_apply_AT(g, v, t);
    for (long i = 0; i < nc; ++i) t[i] = ninv * t[i] - alpha * q[i];
    double beta = sqrt(dot(nc, t, t) / ninv);
    if (!isfinite(beta)) { status = OG_ENAN; goto done; }
    if (beta <= 1e-13 * alpha) { /* breakdown: the Krylov space is exhausted */
      est = 0.0;
      converged = 1;
      break;
    }
    for (long i = 0; i < nc; ++i) q[i] = t[i] / beta;
    /* s = M^-1 (A q - beta M v_k), alpha = ||s||_M */
    og_apply_A(g, q, f);
    for (long i = 0; i < mf; ++i) f[i] -= beta * Mv[i];
    {
      int st = og_pcg(g, mu, eta, f, s, o->inner_tol, o->inner_maxit, &its);
      tot += its;
      if (o->inner_iters) o->inner_iters[solve_idx] = its;
      ++solve_idx;
      if (st != OG_OK) { status = st; goto done; }
    }
    og_apply_M(g, mu, eta, s, y);
    alpha = sqrt(dot(mf, s, y));
    if (!isfinite(alpha) || alpha == 0.0) { status = OG_ENAN; goto done; }
    for (long i = 0; i < mf; ++i) {
      v[i] = s[i] / alpha;
      Mv[i] = y[i] / alpha;
    }
    zeta = -(beta / alpha) * zeta;
    for (long i = 0; i < nc; ++i) {
      d[i] = (q[i] - beta * d[i]) / alpha;
      p[i] -= zeta * d[i];
    }
    for (long i = 0; i < mf; ++i) u[i] += zeta * v[i];
    zs[K] = zeta;
    if (o->zeta) o->zeta[K] = zeta;
    if (o->alpha) o->alpha[K] = alpha;
    if (o->beta) o->beta[K] = beta;
    if (K < o->store_k) {
      memcpy(o->V + (long)K * mf, v, sizeof(double) * mf);
      memcpy(o->Q + (long)K * nc, q, sizeof(double) * nc);
    }
    K += 1;
    sum_all += zeta * zeta;
    /* lower bound over the newest d+1 values zeta_{K-d} .. zeta_K */
    if (K >= o->delay + 1) {
      double win = 0.0;
      for (int j = K - o->delay; j <= K; ++j) {
        win += zs[j - 1] * zs[j - 1];
      }
      est = sqrt(win / sum_all);
      if (o->est_hist) o->est_hist[K - 1] = est;
      if (o->tol > 0.0) {
        if (o->squared_rule ? (win <= o->tol * sum_all) : (est <= o->tol)) converged = 1;
      }
    } else if (o->est_hist) {
      o->est_hist[K - 1] = -1.0;
    }
  }
  if (!converged) status = OG_MAXIT;

finish:
  for (long i = 0; i < mf; ++i) w[i] = (u[i] + w0[i]) * mask[i];
  for (long i = 0; i < nc; ++i)
    if (i == g->pin) p[i] = 0.0;
done:
  if (K_out) *K_out = K;
  if (est_out) *est_out = est;
  if (inner_total) *inner_total = tot;
  free(ghat); free(w0); free(u); free(v); free(Mv); free(s); free(y); free(f);
  free(b); free(q); free(d); free(t); free(mask); free(zs);
  return status;
}

/* ---------------------------------------------------------- saddle residual */

/* res_w = g - W w - A p (unknown faces), res_r = r - A^T w (unpinned cells).
   norms[0] = ||[res_w; res_r]||, [1] = ||res_w||, [2] = ||res_r||,
   [3] = ||[g; r]|| (restricted to unknowns). */
void og_saddle_residual(const og_grid *g, const double *mu, const double *gv,
                        const double *rv, const double *w, const double *p,
                        double *res_w, double *res_r, double *norms) {
  long mf = og_m_full(g), nc = og_n_cells(g);
  double *Ww = malloc(sizeof(double) * mf), *Ap = malloc(sizeof(double) * mf);
  double *mask = malloc(sizeof(double) * mf);
  og_diag_M(g, mu, 0.0, mask);
  og_apply_W(g, mu, w, Ww);
  og_apply_A(g, p, Ap);
  og_apply_AT(g, w, res_r);
  double sw = 0.0, sr = 0.0, sg = 0.0;
  for (long i = 0; i < mf; ++i) {
    double mk = mask[i] > 0.0 ? 1.0 : 0.0;
    res_w[i] = mk * (gv[i] - Ww[i] - Ap[i]);
    sw += res_w[i] * res_w[i];
    sg += mk * gv[i] * gv[i];
  }
  for (long i = 0; i < nc; ++i) {
    double rk = (i == g->pin) ? 0.0 : rv[i];
    res_r[i] = (i == g->pin) ? 0.0 : rk - res_r[i];
    sr += res_r[i] * res_r[i];
    sg += rk * rk;
  }
  norms[0] = sqrt(sw + sr);
  norms[1] = sqrt(sw);
  norms[2] = sqrt(sr);
  norms[3] = sqrt(sg);
  free(Ww);
  free(Ap);
  free(mask);
}
