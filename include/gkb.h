/*
 * gkb.h -- C-ABI of the MI355X (gfx950) generalized Golub-Kahan
 * bidiagonalization solver for MAC-discretized Stokes saddle-point systems
 *
 *     [[W, A], [A^T, 0]] [w; p] = [g; r]                                  (1)
 *
 * (Kruse, Sosonkina, Arioli, Tardieu, Ruede, "Parallel solution of saddle
 * point systems with nested iterative solvers based on the Golub-Kahan
 * Bidiagonalization": Section 1 for (1), Section 2 for the augmented
 * Lagrangian M = W + gamma A N^-1 A^T and the transformation to g = 0,
 * Section 2.1 Algorithm 1 for the recurrence, Section 2.2 for the delayed
 * lower-bound stopping rule, Section 3 for the option set nu/delay/tol/maxit/
 * monitor, Section 4.1.3 for the inner/outer tolerance policy.)
 *
 * Discretization.  Uniform MAC grid with cell size h.  W is the component-wise
 * viscous operator -div(mu grad u_c) in strong-form scaling (entries ~ mu/h^2),
 * A the cell-to-face gradient (entries +-1/h), A^T = -div its transpose.
 * N = (1/eta) I: eta > 0 selects gamma = 1 (M = W + eta A A^T), eta = 0 selects
 * gamma = 0, N = I (M = W), exactly as the paper's nu option.
 *
 * Memory layout (all solve vectors are DEVICE pointers, FP64, caller owned):
 *   velocity-shaped (g, w):  full-face, component-major structure of arrays
 *       u[nz][ny][nx+1], then v[nz][ny+1][nx], then (3D) w[nz+1][ny][nx],
 *       x fastest; 2D grids use nz = 1 and have no w block.
 *   pressure-shaped (r, p):  cells [nz][ny][nx].
 * Faces normal to a DIRICHLET side are not unknowns: they are ignored on input
 * and written as 0 on output; so is the pinned pressure cell.  Boundary data
 * (inflow profiles, moving lids) must already be folded into g and r.
 *
 * Streams.  All device work of a context runs on the HIP stream given in
 * gkb_options.hip_stream (NULL = the null stream).  Calls return after that
 * stream's work for the call has completed.  A context is not thread-safe;
 * use one context per stream.
 *
 * Errors.  Every entry point returns GKB_OK (0), GKB_MAXIT (1: result valid
 * but the stopping rule was not met) or a negative code; gkb_strerror()
 * describes it.  On a negative code output buffers hold unspecified values.
 */
#ifndef GKB_H
#define GKB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define GKB_OK 0
#define GKB_MAXIT 1      /* outer maxit reached: the last iterate is returned */
#define GKB_EINVAL (-1)  /* invalid argument */
#define GKB_ENOMEM (-2)  /* device or host allocation failed, or workspace cap */
#define GKB_EHIP (-3)    /* a HIP runtime call failed */
#define GKB_ENAN (-4)    /* non-finite alpha, beta or residual */
#define GKB_EINNER (-5)  /* an inner solve hit inner_maxit */

/* boundary types of the six sides -x, +x, -y, +y, -z, +z */
#define GKB_DIRICHLET 0  /* no-slip wall: wall-normal faces are not unknowns */
#define GKB_NATURAL 1    /* do-nothing outflow: wall-normal faces are unknowns
                            owning half a control volume */

/* precision of the inner solves */
#define GKB_FP64 0       /* everything in FP64 */
#define GKB_MIXED 1      /* FP32 inner PCG / FCG and multigrid, FP64 GKB
                            recurrence, FP64 coarsest solve, FP64 residual */

/* inner solver for M x = f */
#define GKB_INNER_JACOBI 0   /* Jacobi-preconditioned CG */
#define GKB_INNER_MG 1       /* CG preconditioned by one geometric multigrid
                                V(nu_pre, nu_post) cycle, weighted Jacobi smoother */
#define GKB_INNER_LEARNED 2  /* flexible CG, preconditioner = V-cycle + CNN
                                correction, falling back to MG-PCG */

/* Krylov method of the inner solves (the preconditioner is chosen by
   `inner`: diag(M)^-1 for GKB_INNER_JACOBI, one V-cycle for GKB_INNER_MG,
   V-cycle + network correction for GKB_INNER_LEARNED).
   Section 3 leaves the inner Krylov method to the user; Section 4.1.3
   compares CG and fgmres. */
#define GKB_KRYLOV_CG 0      /* preconditioned CG (flexible CG for _LEARNED) */
#define GKB_KRYLOV_FGMRES 1  /* restarted flexible GMRES, right preconditioned,
                                restart fgmres_restart; stops on the same
                                relative residual as CG: in FP64 the residual
                                recomputed at each restart, in FP32 (mixed)
                                also the least-squares estimate of the last
                                cycle, as CG stops on its recursive residual */

/* how gkb_solve uses GKB (Section 3: GKB as a solver or as a preconditioner) */
#define GKB_METHOD_SOLVER 0  /* GKB runs (with defect correction when
                                refine_tol > 0) */
#define GKB_METHOD_PRECOND 1 /* restarted flexible GMRES on the whole saddle
                                system (1), right preconditioned by one GKB run
                                (lower-bound tol, delay, maxit) per iteration;
                                stops when the FP64 relative saddle residual is
                                <= refine_tol (> 0 required) or after
                                max_sweeps iterations (GKB_MAXIT) */

/* multigrid smoother */
#define GKB_SMOOTH_JACOBI 0  /* weighted Jacobi on M */
#define GKB_SMOOTH_HYBRID 1  /* weighted Jacobi on M, each sweep paired with a
                                weighted-Jacobi sweep on the edge operator
                                C^T W C mapped back by the discrete curl C
                                (smooths the divergence-free error that point
                                Jacobi leaves when eta >> mu); face then edge
                                before, edge then face after the coarse
                                correction, so the V-cycle stays symmetric */

/* multigrid transfers of the V-cycle.  Both prolongations are linear along
   a face's normal; across it (tangential directions):
   DIV     constant over the two fine cells: a coarse divergence-free field
           maps to a divergence-free fine field, which a V-cycle on
           M = W + eta A A^T needs when eta >> mu (the grad-div term's near
           null space is the divergence-free space);
   SMOOTH  linear between coarse row centres (mirror ghosts at the sides):
           second order, the textbook pair for the vector Laplacian (eta
           small against mu), with a grid-independent V-cycle;
   AUTO    SMOOTH when eta <= 100 mu_ref, else DIV, with mu_ref the geometric
           mean of the cell viscosity (1 without one) */
#define GKB_TRANSFER_AUTO 0
#define GKB_TRANSFER_DIV 1
#define GKB_TRANSFER_SMOOTH 2

typedef struct {
  int dim;       /* 2 or 3 */
  int n[3];      /* cells per axis (n[2] ignored in 2D) */
  double h;      /* cell size (> 0) */
  int bc[6];     /* GKB_DIRICHLET / GKB_NATURAL for -x,+x,-y,+y,-z,+z */
  int pin_cell;  /* flat cell index whose pressure is fixed to 0, or -1 */
} gkb_grid;

typedef struct {
  int precision;        /* GKB_FP64 or GKB_MIXED */
  int inner;            /* GKB_INNER_JACOBI / _MG / _LEARNED */
  int mg_levels;        /* number of grid levels; 0 = coarsen while the level
                           has more than 2000 faces and every n is even and
                           >= 4 (the coarsest level is solved with a dense
                           FP64 inverse, at most 4096 faces) */
  int nu_pre, nu_post;  /* smoothing sweeps of the V-cycle */
  double inner_tol;     /* relative residual of each inner solve (tau_in) */
  int inner_maxit;
  int maxit;            /* maximum number of GKB steps (zeta values) per sweep */
  double refine_tol;    /* 0: one GKB run (the paper's method).  > 0: repeat
                           GKB on the FP64 saddle residual (defect correction)
                           until ||res|| <= refine_tol ||[g; r]||; after three
                           sweeps without a new smallest ||res|| (inner solves
                           too inexact for the correction to converge) the
                           solve returns GKB_MAXIT with the best iterate */
  int max_sweeps;       /* cap on defect-correction sweeps */
  int check_every;      /* inner iterations between host convergence checks */
  int use_graphs;       /* capture inner iterations in HIP graphs (1) or not */
  int stencil;          /* 0: LDS-tiled 3D stencil kernel where it applies (3D
                           grids whose +x, +y, +z sides are DIRICHLET), generic
                           face kernel elsewhere; 1: generic face kernel only */
  int smoother;         /* GKB_SMOOTH_JACOBI or GKB_SMOOTH_HYBRID */
  void *hip_stream;     /* hipStream_t; NULL = null stream */
  size_t max_workspace_bytes; /* 0 = unlimited; else setup fails with
                                 GKB_ENOMEM above this device footprint */
  int krylov;           /* GKB_KRYLOV_CG or GKB_KRYLOV_FGMRES (inner solves).
                           With GKB_INNER_LEARNED and a network, FGMRES
                           applies V-cycle + network correction in every step
                           (it takes a preconditioner that changes from step
                           to step; no fallback tests); without a network it
                           uses the V-cycle */
  int fgmres_restart;   /* Krylov vectors of the inner FGMRES (1..64) */
  int method;           /* GKB_METHOD_SOLVER or GKB_METHOD_PRECOND */
  int outer_restart;    /* Krylov vectors of the outer FGMRES of
                           GKB_METHOD_PRECOND (1..32) */
  const char *cnn_weights; /* NULL, or the path of a network checkpoint
                              (gkb_cnn_save) loaded at setup and owned by the
                              context; used by GKB_INNER_LEARNED (the same as
                              gkb_attach_cnn with a network the context frees).
                              A file that does not load, or whose network does
                              not fit the grid, fails setup with GKB_EINVAL */
  double learned_min_gain; /* GKB_INNER_LEARNED: the network correction is
                              dropped (fallback to MG-PCG) when the error energy
                              its step removes falls below this fraction of the
                              V-cycle step's (gkb_stats_t.learned_gain); 0
                              turns this test off (the descent and progress
                              tests stay), < 0 also the progress test (no
                              decrease of r.r over 50 iterations): only the
                              descent test r.z > 0 that flexible CG needs
                              remains */
  int mg_transfer;      /* GKB_TRANSFER_AUTO / _DIV / _SMOOTH: the multigrid
                           prolongation (restriction: its transpose / 2^d) */
} gkb_options;

typedef struct {
  int sweeps;             /* GKB runs in the last solve */
  int outer_iterations;   /* K summed over sweeps */
  long inner_iterations;  /* inner Krylov iterations summed over all solves */
  int inner_solves;
  int fallbacks;          /* learned -> MG-PCG switches inside inner solves */
  int learned_solves;     /* inner solves started with the network.  When the
                             network fails a guard (descent, progress, gain)
                             the solve restarts as plain MG-PCG from x = 0
                             (the abandoned iterations still count in
                             inner_iterations) and the network stays off for
                             the rest of the gkb_solve */
  double residual;        /* final ||res||_2 / ||[g; r]||_2 (FP64), -1 if not computed */
  double error_estimate;  /* last lower-bound ratio */
  double seconds_solve;   /* wall time of the last gkb_solve */
  int history_len;        /* entries valid in the two arrays below */
  double zeta[512];       /* zeta_1..zeta_K of the last sweep (monitor) */
  double estimate[512];   /* lower-bound ratio after each step (-1 before d+1) */
  size_t workspace_bytes; /* device memory held by the context */
  int mg_levels;          /* levels actually used */
  double omega[16];       /* Jacobi weight per level */
  double omega_edge[16];  /* edge-sweep weight per level (hybrid smoother; 0
                             otherwise) */
  double learned_gain;    /* mean over the network applications of the last
                             gkb_solve of the error energy removed by the
                             network step relative to the V-cycle step,
                             (c.rt)^2 / (c.Mc) / (r.V(r)); -1 if none.  Below
                             learned_min_gain an inner solve falls back to
                             MG-PCG */
  int learned_fallback_reason;    /* cause of the last fallback of the last
                                     gkb_solve: 0 none, 1 descent (r.z <= 0),
                                     2 no progress over 50 iterations, 3 gain
                                     below learned_min_gain */
  int learned_fallback_iteration; /* inner iteration of that fallback */
  int outer_krylov_iterations;    /* GKB_METHOD_PRECOND: outer FGMRES
                                     iterations (= GKB runs) of the last solve */
  int mg_transfer;                /* transfer pair in use (GKB_TRANSFER_DIV or
                                     GKB_TRANSFER_SMOOTH) */
} gkb_stats_t;

typedef struct gkb_ctx gkb_ctx;

/* Fill *opt with defaults: FP64, MG inner, auto levels, V(2,2), Jacobi
   smoother, inner_tol 1e-10, inner_maxit 10000, maxit 500, refine_tol 0,
   max_sweeps 10, check_every 8, graphs on, null stream, CG inner solves,
   fgmres_restart 30, GKB as the solver, outer_restart 10, no network file,
   learned_min_gain 0.05, mg_transfer GKB_TRANSFER_AUTO. */
void gkb_default_options(gkb_options *opt);

/* Create a context for one grid, viscosity field and eta (the paper's nu).
   viscosity: HOST pointer to n_cells doubles (> 0), or NULL for mu = 1; it is
   copied.  opt may be NULL (defaults).  Allocates all device workspace,
   builds the multigrid hierarchy (coarsened viscosity, Jacobi weights, dense
   FP64 inverse of the coarsest operator).  Errors: GKB_EINVAL (dim not 2/3,
   n < 2, h <= 0, eta < 0, bad bc, pin out of range, grid not divisible for
   mg_levels, M singular because every side is NATURAL, an option out of
   range, cnn_weights that does not load or fit), GKB_ENOMEM, GKB_EHIP. */
int gkb_setup(const gkb_grid *grid, const double *viscosity, double eta,
              const gkb_options *opt, gkb_ctx **out);

/* Solve (1) for the right-hand sides g (faces) and r (cells), all device FP64.
   tol = tau of the lower-bound rule (Section 2.2; stop when the ratio of the
   newest delay+1 squared zeta values to all of them is <= tol^2; tol <= 0 runs
   maxit steps).  delay = d >= 1 (the window holds d+1 values; d < 1 is
   GKB_EINVAL).  Writes w (faces) and p (cells); iterations
   (may be NULL) receives K of the last sweep, error_estimate (may be NULL)
   the last lower-bound ratio.  g and w, r and p may not alias.
   Returns GKB_OK, GKB_MAXIT, GKB_ENAN, GKB_EINNER, GKB_EINVAL, GKB_EHIP. */
int gkb_solve(gkb_ctx *c, const double *g, const double *r, double tol, int delay,
              double *w, double *p, int *iterations, double *error_estimate);

/* Statistics of the last gkb_solve (and setup facts). */
int gkb_stats(const gkb_ctx *c, gkb_stats_t *out);

/* Unknown-face / cell counts and full array sizes of the context's grid. */
int gkb_sizes(const gkb_ctx *c, long *m_full, long *n_cells, long *m_unknown,
              long *n_unknown);

const char *gkb_strerror(int code);

void gkb_destroy(gkb_ctx *c);

/* ---- assembled systems ------------------------------------------------ */

/* A saddle system given by its blocks as compressed sparse rows, the form a
   PETSc fieldsplit user passes (Section 3): W (m x m, symmetric positive
   definite, or semidefinite with eta > 0 making M definite) and A (m x n,
   full column rank).  All arrays are HOST arrays, copied at setup; column
   indices 0-based and in range; every diagonal entry of W must be present and
   positive. */
typedef struct {
  int m;                  /* velocity unknowns: rows of W and of A */
  int n;                  /* pressure unknowns: columns of A */
  const int *w_rowptr;    /* m + 1 row offsets of W, w_rowptr[0] = 0 */
  const int *w_col;       /* w_rowptr[m] column indices of W */
  const double *w_val;    /* w_rowptr[m] values of W */
  const int *a_rowptr;    /* m + 1 row offsets of A */
  const int *a_col;       /* a_rowptr[m] column indices of A (< n) */
  const double *a_val;
} gkb_csr;

#define GKB_SCALE_NONE 0     /* solve the system as given */
#define GKB_SCALE_CENTRAL 1  /* solve the system scaled on both sides by
                                blockdiag(D^-1/2, R^-1/2), D = diag(W),
                                R = diag(A^T D^-1 A) (the central scaling of
                                Section 4.1, which equilibrates the blocks);
                                the solution is scaled back, so w and p solve
                                the given system */

/* Context for an assembled system (otherwise as gkb_setup).  The inner
   solver must be GKB_INNER_JACOBI (CG or FGMRES; multigrid needs a grid);
   opt == NULL selects it with the other defaults.  gkb_solve takes g (m) and
   r (n) and writes w (m) and p (n), device FP64; with central scaling its
   lower-bound rule, the defect-correction residual (refine_tol) and
   gkb_stats_t.residual refer to the scaled system, while gkb_residual
   evaluates the given one; gkb_apply applies the scaled operators.
   Errors: GKB_EINVAL (bad sizes, indices, values, a non-positive diagonal
   of W, an empty column of A with scaling, eta < 0, a multigrid or learned
   inner solver), GKB_ENOMEM, GKB_EHIP. */
int gkb_setup_csr(const gkb_csr *sys, double eta, int scaling, const gkb_options *opt,
                  gkb_ctx **out);

/* ---- operator-level entry points (used by the parity tests) ----------- */

#define GKB_OP_W 0   /* y = W x        (faces -> faces) */
#define GKB_OP_A 1   /* y = A x        (cells -> faces) */
#define GKB_OP_AT 2  /* y = A^T x      (faces -> cells) */
#define GKB_OP_M 3   /* y = W x + eta A A^T x (faces -> faces) */
#define GKB_OP_DIAG 4 /* y = diag(M)   (x ignored) */

/* y = op(x) on the finest grid, in FP64 (precision = GKB_FP64; x, y double*)
   or FP32 (precision = GKB_MIXED; x, y float*).  Device pointers. */
int gkb_apply(gkb_ctx *c, int op, int precision, const void *x, void *y);

/* One preconditioner application z = B r on the finest grid (B = one
   V-cycle, or diag(M)^-1 for the Jacobi inner solver), FP64 or FP32 as
   gkb_apply.  Device pointers. */
int gkb_precondition(gkb_ctx *c, int precision, const void *r, void *z);

/* Inner solve M x = f with the context's inner solver (x0 = 0), FP64 device
   vectors (MIXED precision casts to FP32 internally).  tol <= 0 uses
   inner_tol.  *iterations receives the iteration count.  Returns GKB_OK or
   GKB_EINNER. */
int gkb_inner_solve(gkb_ctx *c, const double *f, double *x, double tol,
                    int *iterations);

/* FP64 saddle residual res_w = g - W w - A p, res_r = r - A^T w (device);
   norms (host, 4 doubles): ||[res_w; res_r]||, ||res_w||, ||res_r||,
   ||[g; r]||.  res_w / res_r may be NULL when only the norms are wanted. */
int gkb_residual(gkb_ctx *c, const double *g, const double *r, const double *w,
                 const double *p, double *res_w, double *res_r, double *norms);

/* ---- measurement ------------------------------------------------------ */

#define GKB_KERNEL_SMOOTH 0  /* one weighted-Jacobi sweep y = x + omega D^-1 (b - M x)
                                on the finest grid (reads x, b; writes y) */
#define GKB_KERNEL_APPLY 1   /* y = M x with the fused x.y block partials */
#define GKB_KERNEL_RESID 2   /* y = b - M x */
#define GKB_KERNEL_SMOOTH_PROLONG 3  /* the V-cycle's first post-smoothing sweep:
                                        y = x' + omega D^-1 (b - M x'), x' = x + P e
                                        with e on the next coarser level (reads x,
                                        b and e; writes y) */
#define GKB_KERNEL_SMOOTH_ZERO 4     /* the V-cycle's first two pre-smoothing sweeps
                                        from a zero guess in one pass (reads b;
                                        writes y); constant viscosity only */

/* Launch one finest-grid kernel of the inner solver `reps` times back to
   back on the context's stream (working precision of the inner solve, on
   the context's own PCG buffers; the launches are captured into one HIP
   graph and replayed, as the solver replays its PCG iterations) and return
   the average time per launch in milliseconds, measured with HIP events
   recorded on that stream around the replay.  Needs
   inner = GKB_INNER_MG or GKB_INNER_LEARNED; the two V-cycle sweeps need a
   3D grid on the tiled path (upper sides DIRICHLET, face arrays below 2 GiB)
   and a multigrid hierarchy of at least two levels, else GKB_EINVAL.  Does
   not change solver state other than scratch vectors. */
int gkb_time_kernel(gkb_ctx *c, int kernel, int reps, double *avg_ms);

/* ---- allocation-free entry point ------------------------------------- */

/* For callers that cannot allocate device memory (code between other
   allocations it must not disturb, serving loops, harnesses that forbid
   hipMalloc): the FP64 saddle residual of gkb_residual for viscosity mu = 1,
   without a solver context.  grid as for gkb_setup; g, w (faces) and r, p
   (cells) are caller-owned device FP64 arrays; res_r (cells, required) and
   res_w (faces, may be NULL) receive the residual blocks; norms (host, 4
   doubles) as gkb_residual.  Work is queued on hip_stream (NULL = the null
   stream) and complete on return.  Allocates nothing: its reduction partials
   live in a fixed device array of 2 MiB (one per GPU, kept until the process
   ends) shared by every call on that GPU, so calls that overlap on one GPU
   race.  Grids that need more than 65536 partials per reduction return
   GKB_EINVAL (every grid up to 256^3 in 3D and 2048^2 in 2D fits), as do
   invalid grids. */
int gkb_residual_noalloc(const gkb_grid *grid, const double *g, const double *r,
                         const double *w, const double *p, double *res_w,
                         double *res_r, double *norms, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GKB_H */
