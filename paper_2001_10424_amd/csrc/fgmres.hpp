// Restarted flexible GMRES for the inner systems M x = f (right
// preconditioned: the Krylov basis V is built from M z_j with z_j = P(v_j),
// and the correction is formed from the stored z_j, so P may be any fixed or
// varying preconditioner; Saad's flexible variant of GMRES).  The paper
// leaves the inner Krylov method open (Section 3) and compares CG with
// fgmres (Section 4.1.3).
//
// GPU design: the basis is orthogonalised by classical Gram-Schmidt applied
// twice (every coefficient of one pass comes from one multi-vector dot
// kernel, so a step costs a fixed number of launches however long the basis
// is, and the second pass restores the orthogonality one pass loses).  The
// Hessenberg matrix, the Givens rotations and the least-squares right-hand
// side live on the device in FP64 and are updated by one-block kernels, so a
// whole restart cycle is captured in one HIP graph and the host looks at the
// state once per cycle.  Two flags steer the early exits: the solve's
// PcgState (done for good) and a cycle state whose `done` ends the Arnoldi
// steps of the current cycle (converged, breakdown, iteration cap, or the
// cycle is full).
#pragma once
#include "kernels.hpp"

namespace gkb {

constexpr int kGmMaxRestart = 64;  // Krylov vectors per cycle (bound of the option)
constexpr int kGmChunk = 8;        // basis vectors per block row of the dot kernel

struct FgmState {
  double H[kGmMaxRestart + 1][kGmMaxRestart];  // H[i][j]: row i, column j
  double cs[kGmMaxRestart], sn[kGmMaxRestart];  // Givens rotations
  double g[kGmMaxRestart + 1];                  // rotated least-squares rhs
  double y[kGmMaxRestart];                      // solution of the triangular system
  double h[kGmMaxRestart + 1];                  // coefficients of the current pass
  double beta;                                  // ||r|| at the start of the cycle
  int k;                                        // completed Arnoldi steps of the cycle
  int conv;                                     // residual estimate met the tolerance
};

// partials of V_k . w for the basis vectors k in [8 blockIdx.y, +8) of the
// first nv; layout part[k * gridDim.x + blockIdx.x]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gm_mdot(int n, const PcgState* __restrict__ cyc,
                                                    const T* __restrict__ V, long ldv, int nv,
                                                    const T* __restrict__ w,
                                                    double* __restrict__ part) {
  if (cyc->done) return;
  const int k0 = blockIdx.y * kGmChunk;
  const int kn = min(kGmChunk, nv - k0);
  double s[kGmChunk];
#pragma unroll
  for (int q = 0; q < kGmChunk; ++q) s[q] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double wi = double(w[i]);
#pragma unroll
    for (int q = 0; q < kGmChunk; ++q)
      if (q < kn) s[q] += double(V[(k0 + q) * ldv + i]) * wi;
  }
  __shared__ double sh[kBlock / 64];
#pragma unroll
  for (int q = 0; q < kGmChunk; ++q) {
    if (q >= kn) break;  // uniform
    const double t = block_sum<kBlock>(s[q], sh);
    if (threadIdx.x == 0) part[(long)(k0 + q) * gridDim.x + blockIdx.x] = t;
    __syncthreads();
  }
}

// one Gram-Schmidt pass of column j: h = the nv = j+1 coefficient sums
// (fixed order), added to column j of H (pass 0 sets it)
__global__ __launch_bounds__(kFinal) void k_gm_hsum(const PcgState* cyc, FgmState* fs,
                                                    const double* part, int nb, int nv, int j,
                                                    int pass) {
  if (cyc->done) return;
  __shared__ double sh[kFinal / 64];
  for (int k = 0; k < nv; ++k) {
    const double v = sum_partials(part + (long)k * nb, nb, sh);
    if (threadIdx.x == 0) {
      fs->h[k] = v;
      fs->H[k][j] = pass == 0 ? v : fs->H[k][j] + v;
    }
    __syncthreads();
  }
}

// w -= sum_k h_k V_k over the first nv basis vectors; partial w.w
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gm_maxpy(int n, const PcgState* __restrict__ cyc,
                                                     const FgmState* __restrict__ fs,
                                                     const T* __restrict__ V, long ldv, int nv,
                                                     T* __restrict__ w,
                                                     double* __restrict__ part_ww) {
  if (cyc->done) return;
  double ss = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    double wi = double(w[i]);
    for (int k = 0; k < nv; ++k) wi -= fs->h[k] * double(V[k * ldv + i]);
    const T wt = T(wi);
    w[i] = wt;
    ss += double(wt) * double(wt);
  }
  __shared__ double sh[kBlock / 64];
  ss = block_sum<kBlock>(ss, sh);
  if (threadIdx.x == 0) part_ww[blockIdx.x] = ss;
}

// end of Arnoldi step j: H[j+1][j] = ||w||, the earlier rotations applied to
// column j, a new rotation that zeroes H[j+1][j], the rotated right-hand
// side and its last entry |g[j+1]| = the residual norm of the least-squares
// solution; the cycle ends on convergence, breakdown, the iteration cap or
// a full basis
__global__ __launch_bounds__(kFinal) void k_gm_arnoldi_end(PcgState* st, PcgState* cyc,
                                                           FgmState* fs, const double* part_ww,
                                                           int nb, int j, int last) {
  if (cyc->done) return;
  __shared__ double sh[kFinal / 64];
  const double ww = sum_partials(part_ww, nb, sh);
  if (threadIdx.x != 0) return;
  const double hn = sqrt(ww);
  for (int i = 0; i < j; ++i) {
    const double a = fs->H[i][j], b = fs->H[i + 1][j];
    fs->H[i][j] = fs->cs[i] * a + fs->sn[i] * b;
    fs->H[i + 1][j] = -fs->sn[i] * a + fs->cs[i] * b;
  }
  const double a = fs->H[j][j];
  const double rr = sqrt(a * a + hn * hn);
  st->it += 1;
  if (rr == 0.0) {
    // M z_j adds nothing to the basis: the step is dropped, the cycle ends
    // and the next one restarts from the true residual
    fs->k = j;
    cyc->done = 1;
    return;
  }
  const double c = a / rr, s = hn / rr;
  fs->cs[j] = c;
  fs->sn[j] = s;
  fs->H[j][j] = rr;
  fs->H[j + 1][j] = hn;  // kept for the normalisation of v_{j+1}
  fs->g[j + 1] = -s * fs->g[j];
  fs->g[j] = c * fs->g[j];
  fs->k = j + 1;
  const double res2 = fs->g[j + 1] * fs->g[j + 1];
  if (!isfinite(res2) || !isfinite(rr)) {
    st->nonfinite = 1;
    st->status = -4;
    cyc->done = 1;
    return;
  }
  if (res2 <= st->tol2 * st->rr0 || hn == 0.0) {
    fs->conv = 1;
    cyc->done = 1;
  } else if (st->it >= st->maxit || last) {
    cyc->done = 1;
  }
}

// v_{j+1} = w / H[j+1][j]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gm_scale(int n, const PcgState* __restrict__ cyc,
                                                     const FgmState* __restrict__ fs, int j,
                                                     T* __restrict__ v) {
  if (cyc->done) return;
  const T s = T(1.0 / fs->H[j + 1][j]);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) v[i] *= s;
}

// z = dinv v (Jacobi preconditioner)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gm_jacobi(int n, const PcgState* __restrict__ cyc,
                                                      const T* __restrict__ dinv,
                                                      const T* __restrict__ v, T* __restrict__ z) {
  if (cyc->done) return;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) z[i] = dinv[i] * v[i];
}

// back substitution R y = g over the k steps of the cycle (R = the rotated,
// upper triangular H)
__global__ void k_gm_solve_y(const PcgState* st, FgmState* fs) {
  if (st->done || threadIdx.x != 0) return;
  const int k = fs->k;
  for (int i = k - 1; i >= 0; --i) {
    double v = fs->g[i];
    for (int l = i + 1; l < k; ++l) v -= fs->H[i][l] * fs->y[l];
    fs->y[i] = v / fs->H[i][i];
  }
}

// x += sum_{i<k} y_i z_i
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gm_update_x(int n, const PcgState* __restrict__ st,
                                                        const FgmState* __restrict__ fs,
                                                        const T* __restrict__ Z, long ldz,
                                                        T* __restrict__ x) {
  if (st->done) return;
  const int k = fs->k;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    double xi = double(x[i]);
    for (int l = 0; l < k; ++l) xi += fs->y[l] * double(Z[l * ldz + i]);
    x[i] = T(xi);
  }
}

// after the update: done on a non-finite value (-4); convergence and the
// iteration cap are decided on the true residual by the next k_gm_start
__global__ void k_gm_cycle_end(PcgState* st, const FgmState* fs) {
  if (st->done || threadIdx.x != 0) return;
  (void)fs;
  if (st->nonfinite) st->done = 1;
}

// start of a cycle from r (partials of r.r): beta = ||r||, g = beta e_1.
// first = 1 also initialises the solve's state (rr0 = f.f, tolerance,
// iteration cap).  At a restart the recomputed residual decides: done when
// it meets the tolerance (also where the least-squares estimate of the last
// cycle already did: near rounding level the two part), else done with
// status -5 once the iteration cap is reached.  accept_estimate = 1 (FP32
// inner solves) also ends the solve when the last cycle's least-squares
// estimate met the tolerance: that estimate plays the part of CG's
// recursive residual, while f - M x formed in FP32 has a rounding floor
// of about eps_32 |M| |x| / |f|, which on grad-div dominated M (eta >> mu)
// lies above the loose inner tolerances of the mixed-precision solver; the
// FP64 defect correction around the inner solves removes what is left
__global__ __launch_bounds__(kFinal) void k_gm_start(PcgState* st, PcgState* cyc, FgmState* fs,
                                                     const double* part_rr, int nrr, double tol,
                                                     int maxit, int first, int accept_estimate) {
  if (!first && st->done) return;
  __shared__ double sh[kFinal / 64];
  const double rr = sum_partials(part_rr, nrr, sh);
  if (threadIdx.x != 0) return;
  if (first) {
    st->rr0 = rr;
    st->tol2 = tol * tol;
    st->it = 0;
    st->maxit = maxit;
    st->nonfinite = 0;
    st->status = 0;
    st->done = rr == 0.0 ? 1 : 0;
  } else if (!isfinite(rr)) {
    st->nonfinite = 1;
    st->status = -4;
    st->done = 1;
  } else if (rr <= st->tol2 * st->rr0 || (accept_estimate && fs->conv)) {
    st->done = 1;
    st->status = 0;
  } else if (st->it >= st->maxit) {
    st->done = 1;
    st->status = -5;
  }
  st->rr = rr;
  fs->beta = sqrt(rr);
  fs->g[0] = fs->beta;
  for (int i = 1; i <= kGmMaxRestart; ++i) fs->g[i] = 0.0;
  fs->k = 0;
  fs->conv = 0;
  cyc->done = st->done;
}

// v_0 = r / beta
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gm_v0(int n, const PcgState* __restrict__ st,
                                                  const FgmState* __restrict__ fs,
                                                  const T* __restrict__ r, T* __restrict__ v0) {
  if (st->done) return;
  const T s = T(1.0 / fs->beta);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) v0[i] = r[i] * s;
}

}  // namespace gkb
