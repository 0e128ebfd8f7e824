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

/* ------------------------------------------------------ operator bundle */

/* The GKB iteration and its inner solvers see the saddle system only through
   the products with W, A and A^T, the diagonal of M and the masks of the
   unknowns, so the same code serves the matrix-free MAC operators and
   assembled (CSR) matrices. */
typedef struct og_ops og_ops;
struct og_ops {
  long m, n;           /* lengths of the velocity and pressure arrays */
  double eta;          /* M = W + eta A A^T (eta = 0: M = W) */
  const void *data;    /* operator-specific data */
  void (*W)(const og_ops *o, const double *x, double *y);
  void (*A)(const og_ops *o, const double *p, double *y);
  void (*AT)(const og_ops *o, const double *x, double *t);
  void (*diag_M)(const og_ops *o, double *d);
  const double *mask_m; /* 1 on unknown velocity entries, 0 elsewhere */
  const double *mask_n; /* 1 on unknown pressure entries, 0 elsewhere */
};

static void ops_M(const og_ops *o, const double *x, double *y) {
  o->W(o, x, y);
  if (o->eta == 0.0) return;
  double *t = malloc(sizeof(double) * o->n), *z = malloc(sizeof(double) * o->m);
  o->AT(o, x, t);
  o->A(o, t, z);
  for (long f = 0; f < o->m; ++f) y[f] += o->eta * z[f];
  free(t);
  free(z);
}

/* the MAC operators as a bundle */
typedef struct {
  const og_grid *g;
  const double *mu;
} mac_data;

static void mac_W(const og_ops *o, const double *x, double *y) {
  const mac_data *d = o->data;
  og_apply_W(d->g, d->mu, x, y);
}
static void mac_A(const og_ops *o, const double *p, double *y) {
  og_apply_A(((const mac_data *)o->data)->g, p, y);
}
static void mac_AT(const og_ops *o, const double *x, double *t) {
  og_apply_AT(((const mac_data *)o->data)->g, x, t);
}
static void mac_diag(const og_ops *o, double *d) {
  const mac_data *md = o->data;
  og_diag_M(md->g, md->mu, o->eta, d);
}

/* fills *o for the MAC grid; the masks are allocated (free with
   mac_ops_free) */
static int mac_ops(og_ops *o, mac_data *md, const og_grid *g, const double *mu, double eta) {
  md->g = g;
  md->mu = mu;
  o->m = og_m_full(g);
  o->n = og_n_cells(g);
  o->eta = eta;
  o->data = md;
  o->W = mac_W;
  o->A = mac_A;
  o->AT = mac_AT;
  o->diag_M = mac_diag;
  double *mm = malloc(sizeof(double) * o->m), *mn = malloc(sizeof(double) * o->n);
  if (!mm || !mn) {
    free(mm);
    free(mn);
    return OG_ENOMEM;
  }
  /* unknown faces: the diagonal of W is positive exactly there */
  og_diag_M(g, mu, 0.0, mm);
  for (long i = 0; i < o->m; ++i) mm[i] = mm[i] > 0.0 ? 1.0 : 0.0;
  for (long i = 0; i < o->n; ++i) mn[i] = (i == g->pin) ? 0.0 : 1.0;
  o->mask_m = mm;
  o->mask_n = mn;
  return OG_OK;
}

static void mac_ops_free(og_ops *o) {
  free((void *)o->mask_m);
  free((void *)o->mask_n);
}

/* ------------------------------------------------------ inner solvers */

/* Solve M x = f by CG with the Jacobi preconditioner diag(M)^-1, x0 = 0.
   Stops when ||f - M x_i||_2 <= tol ||f||_2 (recursive residual) or after
   maxit iterations.  Returns OG_OK or OG_EINNER; *iters = iterations done. */
static int pcg_ops(const og_ops *o, const double *f, double *x, double tol, int maxit,
                   int *iters) {
  long mf = o->m;
  double *r = malloc(sizeof(double) * mf), *z = malloc(sizeof(double) * mf);
  double *p = malloc(sizeof(double) * mf), *q = malloc(sizeof(double) * mf);
  double *dg = malloc(sizeof(double) * mf);
  if (!r || !z || !p || !q || !dg) return OG_ENOMEM;
  o->diag_M(o, dg);
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
    ops_M(o, p, q);
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

int og_pcg(const og_grid *g, const double *mu, double eta, const double *f, double *x,
           double tol, int maxit, int *iters) {
  og_ops o;
  mac_data md;
  if (mac_ops(&o, &md, g, mu, eta) != OG_OK) return OG_ENOMEM;
  int st = pcg_ops(&o, f, x, tol, maxit, iters);
  mac_ops_free(&o);
  return st;
}

/* Flexible GMRES (Saad 1993) for M x = f, x0 = 0, restarted after `restart`
   steps, with the Jacobi preconditioner applied on the right: z_j =
   diag(M)^-1 v_j, basis vectors from M z_j orthogonalised by modified
   Gram-Schmidt, Givens rotations on the Hessenberg matrix, x += Z y at the
   end of a cycle (early when the residual norm of the least-squares problem
   is <= tol ||f||) and a restart from the true residual.  Stops when the
   true residual at the end of a cycle is <= tol ||f||, or after maxit steps
   (OG_EINNER). */
static int fgmres_ops(const og_ops *o, const double *f, double *x, double tol, int restart,
                      int maxit, int *iters) {
  long mf = o->m;
  int R = restart;
  double *V = malloc(sizeof(double) * mf * (R + 1)), *Z = malloc(sizeof(double) * mf * R);
  double *H = calloc((size_t)(R + 1) * R, sizeof(double));
  double *cs = malloc(sizeof(double) * R), *sn = malloc(sizeof(double) * R);
  double *gv = malloc(sizeof(double) * (R + 1)), *y = malloc(sizeof(double) * R);
  double *dg = malloc(sizeof(double) * mf), *r = malloc(sizeof(double) * mf);
  if (!V || !Z || !H || !cs || !sn || !gv || !y || !dg || !r) return OG_ENOMEM;
  o->diag_M(o, dg);
  for (long i = 0; i < mf; ++i) {
    x[i] = 0.0;
    r[i] = f[i];
  }
  double ff = dot(mf, f, f);
  int it = 0, status = OG_EINNER;
  if (ff == 0.0) status = OG_OK;
  while (status == OG_EINNER) {
    double beta = sqrt(dot(mf, r, r));
    if (!isfinite(beta)) {
      status = OG_ENAN;
      break;
    }
    if (beta * beta <= tol * tol * ff) {
      status = OG_OK;
      break;
    }
    if (it >= maxit) break;
    for (long i = 0; i < mf; ++i) V[i] = r[i] / beta;
    for (int i = 0; i <= R; ++i) gv[i] = 0.0;
    gv[0] = beta;
    int k = 0, conv = 0;
    for (int j = 0; j < R && it < maxit; ++j) {
      double *vj = V + (long)j * mf, *zj = Z + (long)j * mf, *w = V + (long)(j + 1) * mf;
      for (long i = 0; i < mf; ++i) zj[i] = dg[i] > 0.0 ? vj[i] / dg[i] : 0.0;
      ops_M(o, zj, w);
      for (int i = 0; i <= j; ++i) {
        double hij = dot(mf, w, V + (long)i * mf);
        H[(long)i * R + j] = hij;
        for (long l = 0; l < mf; ++l) w[l] -= hij * V[(long)i * mf + l];
      }
      double hn = sqrt(dot(mf, w, w));
      for (int i = 0; i < j; ++i) { /* earlier rotations on column j */
        double a = H[(long)i * R + j], b = H[(long)(i + 1) * R + j];
        H[(long)i * R + j] = cs[i] * a + sn[i] * b;
        H[(long)(i + 1) * R + j] = -sn[i] * a + cs[i] * b;
      }
      double a = H[(long)j * R + j], rr = sqrt(a * a + hn * hn);
      ++it;
      if (rr == 0.0) break; /* M z_j adds nothing: restart */
      cs[j] = a / rr;
      sn[j] = hn / rr;
      H[(long)j * R + j] = rr;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      k = j + 1;
      if (gv[j + 1] * gv[j + 1] <= tol * tol * ff || hn == 0.0) {
        conv = 1;
        break;
      }
      for (long l = 0; l < mf; ++l) w[l] /= hn;
    }
    for (int i = k - 1; i >= 0; --i) { /* R y = g */
      double v = gv[i];
      for (int l = i + 1; l < k; ++l) v -= H[(long)i * R + l] * y[l];
      y[i] = v / H[(long)i * R + i];
    }
    for (int l = 0; l < k; ++l)
      for (long i = 0; i < mf; ++i) x[i] += y[l] * Z[(long)l * mf + i];
    /* the true residual decides, also after the estimate met the tolerance
       (near rounding level the two part) */
    (void)conv;
    ops_M(o, x, r);
    for (long i = 0; i < mf; ++i) r[i] = f[i] - r[i];
  }
  if (iters) *iters = it;
  free(V); free(Z); free(H); free(cs); free(sn); free(gv); free(y); free(dg); free(r);
  return status;
}

/* ---------------------------------------------------------------- GKB */

typedef struct {
  double tol;         /* tau of the lower-bound rule; <= 0 runs to maxit */
  int delay;          /* d */
  int maxit;          /* maximum number of zeta values (K) */
  double inner_tol;   /* relative residual of each inner solve */
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
  int inner_krylov;   /* 0: Jacobi-PCG, 1: FGMRES with Jacobi on the right */
  int restart;        /* FGMRES restart (<= 0: 30) */
} og_gkb_opts;

/* working state of one GKB run: the newest bidiagonalization vectors and
   coefficients (generalized Golub-Kahan relations A Q = M V B,
   A^T V = N Q B^T with V^T M V = I, Q^T N Q = I, Section 2.1) and the
   Craig-variant iterates built from them */
typedef struct {
  const og_ops *o;
  const og_gkb_opts *opt;
  double ninv;            /* N^-1 = ninv I: eta for eta > 0, else 1 */
  double *v, *Mv, *s, *y; /* velocity: v_k, M v_k, inner solution, M s */
  double *f;              /* inner right-hand side */
  double *q, *t;          /* pressure: q_k, unnormalised next q */
  double alpha, beta;     /* alpha_k, beta_k */
  double *u, *d, *p;      /* Craig iterates: u_k, direction d_k, p_k */
  double zeta;
  int solves, inner_total;
} gk_state;

static int gk_inner(gk_state *S, const double *f, double *x) {
  int its = 0, st;
  const og_gkb_opts *o = S->opt;
  if (o->inner_krylov == 1)
    st = fgmres_ops(S->o, f, x, o->inner_tol, o->restart > 0 ? o->restart : 30, o->inner_maxit,
                    &its);
  else
    st = pcg_ops(S->o, f, x, o->inner_tol, o->inner_maxit, &its);
  S->inner_total += its;
  if (o->inner_iters) o->inner_iters[S->solves] = its;
  S->solves += 1;
  return st;
}

/* v = s / ||s||_M and M v from the inner solution s (alpha = ||s||_M by an
   explicit product with M) */
static int gk_normalise_v(gk_state *S) {
  long m = S->o->m;
  ops_M(S->o, S->s, S->y);
  S->alpha = sqrt(dot(m, S->s, S->y));
  if (!isfinite(S->alpha) || S->alpha == 0.0) return OG_ENAN;
  for (long i = 0; i < m; ++i) {
    S->v[i] = S->s[i] / S->alpha;
    S->Mv[i] = S->y[i] / S->alpha;
  }
  return OG_OK;
}

/* first column of the bidiagonalization from b = r - A^T w0:
   beta_1 = ||b||_{N^-1}, q_1 = N^-1 b / beta_1, M s = A q_1, alpha_1, v_1 */
static int gk_first(gk_state *S, const double *b, double beta1) {
  long n = S->o->n;
  S->beta = beta1;
  for (long i = 0; i < n; ++i) S->q[i] = S->ninv * b[i] / beta1;
  S->o->A(S->o, S->q, S->f);
  int st = gk_inner(S, S->f, S->s);
  if (st != OG_OK) return st;
  return gk_normalise_v(S);
}

/* next column: from A^T V = N Q B^T, beta_{k+1} N q_{k+1} = A^T v_k -
   alpha_k N q_k, i.e. t = N^-1 A^T v_k - alpha_k q_k, beta = ||t||_N; from
   A Q = M V B, alpha_{k+1} M v_{k+1} = A q_{k+1} - beta_{k+1} M v_k, solved
   with the inner solver.  *breakdown = 1 when beta is at rounding level
   (the Krylov space is exhausted). */
static int gk_next(gk_state *S, int *breakdown) {
  long m = S->o->m, n = S->o->n;
  S->o->AT(S->o, S->v, S->t);
  for (long i = 0; i < n; ++i) S->t[i] = S->ninv * S->t[i] - S->alpha * S->q[i];
  double beta = sqrt(dot(n, S->t, S->t) / S->ninv);
  if (!isfinite(beta)) return OG_ENAN;
  *breakdown = beta <= 1e-13 * S->alpha;
  if (*breakdown) return OG_OK;
  S->beta = beta;
  for (long i = 0; i < n; ++i) S->q[i] = S->t[i] / beta;
  S->o->A(S->o, S->q, S->f);
  for (long i = 0; i < m; ++i) S->f[i] -= beta * S->Mv[i];
  int st = gk_inner(S, S->f, S->s);
  if (st != OG_OK) return st;
  return gk_normalise_v(S);
}

/* Craig-variant update with the newest column: zeta_k = beta_1 / alpha_1
   at the first step, then -(beta_k / alpha_k) zeta_{k-1};
   d_k = (q_k - beta_k d_{k-1}) / alpha_k; u_k = u_{k-1} + zeta_k v_k,
   p_k = p_{k-1} - zeta_k d_k */
static void craig_update(gk_state *S, int first) {
  long m = S->o->m, n = S->o->n;
  S->zeta = first ? S->beta / S->alpha : -(S->beta / S->alpha) * S->zeta;
  for (long i = 0; i < n; ++i) {
    S->d[i] = first ? S->q[i] / S->alpha : (S->q[i] - S->beta * S->d[i]) / S->alpha;
    S->p[i] = first ? -S->zeta * S->d[i] : S->p[i] - S->zeta * S->d[i];
  }
  for (long i = 0; i < m; ++i) S->u[i] = first ? S->zeta * S->v[i] : S->u[i] + S->zeta * S->v[i];
}

/* lower bound of the energy-norm error relative to the solution, from the
   newest delay+1 zeta values (Section 2.2); returns -1 before K = d+1 */
static double lower_bound_ratio(const double *zs, int K, int delay, double sum_all,
                                double *window) {
  if (K < delay + 1) return -1.0;
  double win = 0.0;
  for (int j = K - delay; j <= K; ++j) win += zs[j - 1] * zs[j - 1];
  *window = win;
  return sqrt(win / sum_all);
}

/* One GKB run for [[W, A], [A^T, 0]] [w; p] = [g; r] on an operator bundle:
   the transformation to a zero first right-hand side (Section 2: with
   ghat = g + gamma A N^-1 r, w0 = M^-1 ghat, u = w - w0 solves the system
   with right-hand side [0; b], b = r - A^T w0), the bidiagonalization with
   the Craig-variant iterates, and the delayed lower-bound stopping rule. */
static int gkb_run_ops(const og_ops *o, const double *gv, const double *rv,
                       const og_gkb_opts *opt, double *w, double *p, int *K_out,
                       double *est_out, int *inner_total) {
  long mf = o->m, nc = o->n;
  if (o->eta < 0.0 || opt->delay < 0 || opt->maxit < 1) return OG_EINVAL;
  gk_state S;
  memset(&S, 0, sizeof(S));
  S.o = o;
  S.opt = opt;
  S.ninv = o->eta > 0.0 ? o->eta : 1.0;
  double *ghat = calloc(mf, sizeof(double)), *w0 = calloc(mf, sizeof(double));
  double *b = calloc(nc, sizeof(double)), *zs = calloc(opt->maxit + 1, sizeof(double));
  S.v = calloc(mf, sizeof(double));
  S.Mv = calloc(mf, sizeof(double));
  S.s = calloc(mf, sizeof(double));
  S.y = calloc(mf, sizeof(double));
  S.f = calloc(mf, sizeof(double));
  S.u = calloc(mf, sizeof(double));
  S.q = calloc(nc, sizeof(double));
  S.t = calloc(nc, sizeof(double));
  S.d = calloc(nc, sizeof(double));
  S.p = p;
  int status = OG_OK, K = 0;
  double est = 1.0;

  /* transformation */
  for (long i = 0; i < mf; ++i) ghat[i] = gv[i] * o->mask_m[i];
  if (o->eta > 0.0) {
    double *rr = malloc(sizeof(double) * nc), *Ar = malloc(sizeof(double) * mf);
    for (long i = 0; i < nc; ++i) rr[i] = rv[i] * o->mask_n[i];
    o->A(o, rr, Ar);
    for (long i = 0; i < mf; ++i) ghat[i] += o->eta * Ar[i];
    free(rr);
    free(Ar);
  }
  if (!all_zero(mf, ghat)) {
    int st = gk_inner(&S, ghat, w0);
    if (st != OG_OK) { status = st; goto done; }
  } else {
    S.solves = 1;
  }
  o->AT(o, w0, b);
  for (long i = 0; i < nc; ++i) b[i] = rv[i] * o->mask_n[i] - b[i];

  double beta1 = sqrt(S.ninv * dot(nc, b, b));
  for (long i = 0; i < nc; ++i) p[i] = 0.0;
  if (beta1 == 0.0) {
    est = 0.0;
    goto finish;
  }
  {
    int st = gk_first(&S, b, beta1);
    if (st != OG_OK) { status = st; goto done; }
  }
  int converged = 0;
  double sum_all = 0.0;
  for (;;) {
    craig_update(&S, K == 0);
    zs[K] = S.zeta;
    if (opt->zeta) opt->zeta[K] = S.zeta;
    if (opt->alpha) opt->alpha[K] = S.alpha;
    if (opt->beta) opt->beta[K] = S.beta;
    if (K < opt->store_k) {
      memcpy(opt->V + (long)K * mf, S.v, sizeof(double) * mf);
      memcpy(opt->Q + (long)K * nc, S.q, sizeof(double) * nc);
    }
    K += 1;
    sum_all += S.zeta * S.zeta;
    double win = 0.0;
    double e = lower_bound_ratio(zs, K, opt->delay, sum_all, &win);
    if (opt->est_hist) opt->est_hist[K - 1] = e;
    if (e >= 0.0) {
      est = e;
      if (opt->tol > 0.0 && (opt->squared_rule ? (win <= opt->tol * sum_all) : (e <= opt->tol))) {
        converged = 1;
        break;
      }
    }
    if (K >= opt->maxit) break;
    int breakdown = 0;
    int st = gk_next(&S, &breakdown);
    if (st != OG_OK) { status = st; goto done; }
    if (breakdown) {
      est = 0.0;
      converged = 1;
      break;
    }
  }
  if (!converged) status = OG_MAXIT;

finish:
  for (long i = 0; i < mf; ++i) w[i] = (S.u[i] + w0[i]) * o->mask_m[i];
  for (long i = 0; i < nc; ++i) p[i] *= o->mask_n[i];
done:
  if (K_out) *K_out = K;
  if (est_out) *est_out = est;
  if (inner_total) *inner_total = S.inner_total;
  free(ghat); free(w0); free(b); free(zs);
  free(S.v); free(S.Mv); free(S.s); free(S.y); free(S.f); free(S.u);
  free(S.q); free(S.t); free(S.d);
  return status;
}

/* Solve [[W, A], [A^T, 0]] [w; p] = [g; r] on the MAC grid.  Returns OG_OK,
   OG_MAXIT or an error; *K = number of zeta values computed, *est = last
   lower-bound ratio. */
int og_gkb_solve(const og_grid *g, const double *mu, double eta, const double *gv,
                 const double *rv, const og_gkb_opts *o, double *w, double *p,
                 int *K_out, double *est_out, int *inner_total) {
  og_ops ops;
  mac_data md;
  if (eta < 0.0 || o->delay < 0 || o->maxit < 1) return OG_EINVAL;
  if (mac_ops(&ops, &md, g, mu, eta) != OG_OK) return OG_ENOMEM;
  int st = gkb_run_ops(&ops, gv, rv, o, w, p, K_out, est_out, inner_total);
  mac_ops_free(&ops);
  return st;
}

/* ------------------------------------------- GKB as a preconditioner */

/* y = K x for the saddle matrix K = [[W, A], [A^T, 0]] on the unknowns;
   x, y: velocity block then pressure block */
static void saddle_apply(const og_ops *o, const double *x, double *y) {
  long m = o->m, n = o->n;
  double *Ap = malloc(sizeof(double) * m);
  double *xp = malloc(sizeof(double) * n);
  for (long i = 0; i < n; ++i) xp[i] = x[m + i] * o->mask_n[i];
  o->W(o, x, y);
  o->A(o, xp, Ap);
  for (long i = 0; i < m; ++i) y[i] = (y[i] + Ap[i]) * o->mask_m[i];
  o->AT(o, x, y + m);
  for (long i = 0; i < n; ++i) y[m + i] *= o->mask_n[i];
  free(Ap);
  free(xp);
}

/* Flexible GMRES (restart `restart`, modified Gram-Schmidt, Givens
   rotations) on the whole saddle system, right preconditioned by one GKB run
   per step (the GKB options of `gopt`); Section 3 offers GKB as a solver or
   as a preconditioner.  Stops when the residual norm of the least-squares
   problem, or the true residual at a restart, is <= tol ||[g; r]||, or after
   maxit steps (OG_MAXIT).  *iters: outer steps (= GKB runs). */
static int gkb_fgmres_ops(const og_ops *o, const double *gv, const double *rv,
                          const og_gkb_opts *gopt, double tol, int restart, int maxit,
                          double *w, double *p, int *iters, int *inner_total) {
  long m = o->m, n = o->n, N = m + n;
  int R = restart;
  double *V = malloc(sizeof(double) * N * (R + 1)), *Z = malloc(sizeof(double) * N * R);
  double *H = calloc((size_t)(R + 1) * R, sizeof(double));
  double *cs = malloc(sizeof(double) * R), *sn = malloc(sizeof(double) * R);
  double *gr = malloc(sizeof(double) * (R + 1)), *y = malloc(sizeof(double) * R);
  double *bb = malloc(sizeof(double) * N), *x = calloc(N, sizeof(double));
  double *r = malloc(sizeof(double) * N);
  for (long i = 0; i < m; ++i) bb[i] = gv[i] * o->mask_m[i];
  for (long i = 0; i < n; ++i) bb[m + i] = rv[i] * o->mask_n[i];
  memcpy(r, bb, sizeof(double) * N);
  double bnorm2 = dot(N, bb, bb);
  int it = 0, status = OG_MAXIT, tot = 0;
  for (;;) {
    double beta = sqrt(dot(N, r, r));
    if (!isfinite(beta)) { status = OG_ENAN; break; }
    if (beta * beta <= tol * tol * bnorm2) { status = OG_OK; break; }
    if (it >= maxit) break;
    for (long i = 0; i < N; ++i) V[i] = r[i] / beta;
    for (int i = 0; i <= R; ++i) gr[i] = 0.0;
    gr[0] = beta;
    int k = 0, conv = 0, err = OG_OK;
    for (int j = 0; j < R && it < maxit; ++j) {
      double *vj = V + (long)j * N, *zj = Z + (long)j * N, *wv = V + (long)(j + 1) * N;
      int K = 0, its = 0;
      double est = 0.0;
      int st = gkb_run_ops(o, vj, vj + m, gopt, zj, zj + m, &K, &est, &its);
      tot += its;
      if (st < 0) { err = st; break; }
      saddle_apply(o, zj, wv);
      for (int i = 0; i <= j; ++i) {
        double hij = dot(N, wv, V + (long)i * N);
        H[(long)i * R + j] = hij;
        for (long l = 0; l < N; ++l) wv[l] -= hij * V[(long)i * N + l];
      }
      double hn = sqrt(dot(N, wv, wv));
      for (int i = 0; i < j; ++i) {
        double a = H[(long)i * R + j], b = H[(long)(i + 1) * R + j];
        H[(long)i * R + j] = cs[i] * a + sn[i] * b;
        H[(long)(i + 1) * R + j] = -sn[i] * a + cs[i] * b;
      }
      double a = H[(long)j * R + j], rr = sqrt(a * a + hn * hn);
      ++it;
      if (rr == 0.0) break;
      cs[j] = a / rr;
      sn[j] = hn / rr;
      H[(long)j * R + j] = rr;
      gr[j + 1] = -sn[j] * gr[j];
      gr[j] = cs[j] * gr[j];
      k = j + 1;
      if (gr[j + 1] * gr[j + 1] <= tol * tol * bnorm2 || hn == 0.0) { conv = 1; break; }
      for (long l = 0; l < N; ++l) wv[l] /= hn;
    }
    if (err != OG_OK) { status = err; break; }
    for (int i = k - 1; i >= 0; --i) {
      double v = gr[i];
      for (int l = i + 1; l < k; ++l) v -= H[(long)i * R + l] * y[l];
      y[i] = v / H[(long)i * R + i];
    }
    for (int l = 0; l < k; ++l)
      for (long i = 0; i < N; ++i) x[i] += y[l] * Z[(long)l * N + i];
    if (conv) { status = OG_OK; break; }
    saddle_apply(o, x, r);
    for (long i = 0; i < N; ++i) r[i] = bb[i] - r[i];
  }
  for (long i = 0; i < m; ++i) w[i] = x[i] * o->mask_m[i];
  for (long i = 0; i < n; ++i) p[i] = x[m + i] * o->mask_n[i];
  if (iters) *iters = it;
  if (inner_total) *inner_total = tot;
  free(V); free(Z); free(H); free(cs); free(sn); free(gr); free(y); free(bb); free(x); free(r);
  return status;
}

int og_gkb_fgmres(const og_grid *g, const double *mu, double eta, const double *gv,
                  const double *rv, const og_gkb_opts *o, double tol, int restart, int maxit,
                  double *w, double *p, int *iters, int *inner_total) {
  og_ops ops;
  mac_data md;
  if (eta < 0.0 || restart < 1 || maxit < 1 || !(tol > 0.0)) return OG_EINVAL;
  if (mac_ops(&ops, &md, g, mu, eta) != OG_OK) return OG_ENOMEM;
  int st = gkb_fgmres_ops(&ops, gv, rv, o, tol, restart, maxit, w, p, iters, inner_total);
  mac_ops_free(&ops);
  return st;
}

/* --------------------------------------------------- assembled (CSR) system */

/* a saddle system given by CSR blocks W (m x m) and A (m x n) */
typedef struct {
  const int *wp, *wc;
  const double *wv;
  const int *ap, *ac;
  const double *av;
} csr_data;

static void csr_W(const og_ops *o, const double *x, double *y) {
  const csr_data *d = o->data;
  for (long i = 0; i < o->m; ++i) {
    double acc = 0.0;
    for (int e = d->wp[i]; e < d->wp[i + 1]; ++e) acc += d->wv[e] * x[d->wc[e]];
    y[i] = acc;
  }
}
static void csr_A(const og_ops *o, const double *p, double *y) {
  const csr_data *d = o->data;
  for (long i = 0; i < o->m; ++i) {
    double acc = 0.0;
    for (int e = d->ap[i]; e < d->ap[i + 1]; ++e) acc += d->av[e] * p[d->ac[e]];
    y[i] = acc;
  }
}
static void csr_AT(const og_ops *o, const double *x, double *t) {
  const csr_data *d = o->data;
  for (long k = 0; k < o->n; ++k) t[k] = 0.0;
  for (long i = 0; i < o->m; ++i)
    for (int e = d->ap[i]; e < d->ap[i + 1]; ++e) t[d->ac[e]] += d->av[e] * x[i];
}
static void csr_diag(const og_ops *o, double *dg) {
  const csr_data *d = o->data;
  for (long i = 0; i < o->m; ++i) {
    double w = 0.0, a = 0.0;
    for (int e = d->wp[i]; e < d->wp[i + 1]; ++e)
      if (d->wc[e] == i) w += d->wv[e];
    for (int e = d->ap[i]; e < d->ap[i + 1]; ++e) a += d->av[e] * d->av[e];
    dg[i] = w + o->eta * a;
  }
}

/* central scaling of Section 4.1: sw = diag(W)^-1/2 (m), sp = diag(A^T
   diag(W)^-1 A)^-1/2 (n).  Returns OG_EINVAL for a non-positive diagonal
   entry of W or an empty column of A. */
int og_csr_central_scaling(int m, int n, const int *wp, const int *wc, const double *wv,
                           const int *ap, const int *ac, const double *av, double *sw,
                           double *sp) {
  for (int i = 0; i < m; ++i) {
    double dw = 0.0;
    for (int e = wp[i]; e < wp[i + 1]; ++e)
      if (wc[e] == i) dw += wv[e];
    if (!(dw > 0.0)) return OG_EINVAL;
    sw[i] = dw; /* D for now */
  }
  for (int k = 0; k < n; ++k) sp[k] = 0.0;
  for (int i = 0; i < m; ++i)
    for (int e = ap[i]; e < ap[i + 1]; ++e) sp[ac[e]] += av[e] * av[e] / sw[i];
  for (int k = 0; k < n; ++k) {
    if (!(sp[k] > 0.0)) return OG_EINVAL;
    sp[k] = 1.0 / sqrt(sp[k]);
  }
  for (int i = 0; i < m; ++i) sw[i] = 1.0 / sqrt(sw[i]);
  return OG_OK;
}

/* GKB on an assembled system, optionally centrally scaled: the scaled
   blocks S_w W S_w and S_w A S_p are formed explicitly, GKB solves the
   scaled system for the right-hand sides S_w g, S_p r, and the solution is
   scaled back, w = S_w w', p = S_p p' (the scaling changes the iterates, not
   the solution of the system). */
int og_gkb_solve_csr(int m, int n, const int *wp, const int *wc, const double *wv,
                     const int *ap, const int *ac, const double *av, double eta, int scaling,
                     const double *gv, const double *rv, const og_gkb_opts *opt, double *w,
                     double *p, int *K_out, double *est_out, int *inner_total) {
  if (m < 1 || n < 1 || eta < 0.0 || opt->delay < 0 || opt->maxit < 1) return OG_EINVAL;
  long nw = wp[m], na = ap[m];
  double *sw = malloc(sizeof(double) * m), *sp = malloc(sizeof(double) * n);
  double *wsc = malloc(sizeof(double) * (nw > 0 ? nw : 1));
  double *asc = malloc(sizeof(double) * (na > 0 ? na : 1));
  double *gs = malloc(sizeof(double) * m), *rs = malloc(sizeof(double) * n);
  double *mm = malloc(sizeof(double) * m), *mn = malloc(sizeof(double) * n);
  int st = OG_OK;
  if (scaling) {
    st = og_csr_central_scaling(m, n, wp, wc, wv, ap, ac, av, sw, sp);
  } else {
    for (int i = 0; i < m; ++i) sw[i] = 1.0;
    for (int k = 0; k < n; ++k) sp[k] = 1.0;
  }
  if (st == OG_OK) {
    for (int i = 0; i < m; ++i)
      for (int e = wp[i]; e < wp[i + 1]; ++e) wsc[e] = sw[i] * wv[e] * sw[wc[e]];
    for (int i = 0; i < m; ++i)
      for (int e = ap[i]; e < ap[i + 1]; ++e) asc[e] = sw[i] * av[e] * sp[ac[e]];
    for (int i = 0; i < m; ++i) {
      gs[i] = sw[i] * gv[i];
      mm[i] = 1.0;
    }
    for (int k = 0; k < n; ++k) {
      rs[k] = sp[k] * rv[k];
      mn[k] = 1.0;
    }
    csr_data d = {wp, wc, wsc, ap, ac, asc};
    og_ops o = {m, n, eta, &d, csr_W, csr_A, csr_AT, csr_diag, mm, mn};
    st = gkb_run_ops(&o, gs, rs, opt, w, p, K_out, est_out, inner_total);
    for (int i = 0; i < m; ++i) w[i] *= sw[i];
    for (int k = 0; k < n; ++k) p[k] *= sp[k];
  }
  free(sw); free(sp); free(wsc); free(asc); free(gs); free(rs); free(mm); free(mn);
  return st;
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
