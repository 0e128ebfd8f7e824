// HIP kernels for gfx950: MAC operators with fused reductions, BLAS-1
// updates of the GKB recurrence and of PCG, multigrid transfers and the dense
// FP64 coarsest-grid solve.
//
// Reductions are deterministic: each block reduces its values with a fixed
// wave-shuffle tree and a fixed-order pass over the waves, writes one FP64
// partial, and a one-block kernel sums the partials in a fixed order.
#pragma once
#include <hip/hip_runtime.h>

#include "mac.hpp"

namespace gkb {

constexpr int kBlock = 256;   // threads per block (4 wave64)
constexpr int kFinal = 1024;  // threads of the one-block finalisers

// ------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum, result valid in thread 0; fixed order
template <int BS>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) s += sh[w];
  }
  return s;
}

// Sum of n partials in a fixed order (one block of kFinal threads): each
// thread's strided share, then the block sum.
__device__ __forceinline__ double thread_partials(const double* __restrict__ part, int n) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += kFinal) v += part[i];
  return v;
}
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n, double* sh) {
  return block_sum<kFinal>(thread_partials(part, n), sh);  // valid in thread 0
}

__global__ __launch_bounds__(kFinal) void k_sum_partials(const double* part, int n, double* out) {
  __shared__ double sh[kFinal / 64];
  double s = sum_partials(part, n, sh);
  if (threadIdx.x == 0) *out = s;
}

// ------------------------------------------------------------ PCG state

struct PcgState {
  double rz, pq, alpha, beta, rr, rr0, tol2;
  double rz_prev;   // flexible CG
  double rt2;       // squared norm of the post-V-cycle residual (learned path)
  double theta;     // energy-optimal weight of the network correction
  double gain;      // error energy removed by that step, (c.rt)^2 / (c.Mc)
  double gain_sum;  // sum over network applications of gain / (r.V(r))
  double ring[10];  // r.r sampled every 5 iterations (stagnation test)
  int it, maxit, done, status, nonfinite;
  int fallback;     // learned preconditioner switched off for this solve
  int stagnant;     // no decrease of r.r over the last 50 iterations
  int use_zv;       // direction from the V-cycle alone
  int fallbacks;
  int fb_it;        // iteration and cause of the fallback (1 descent,
  int fb_reason;    // 2 stagnation, 3 gain below the threshold)
  int gain_n;       // network applications counted in gain_sum
};

// ------------------------------------------------- face-operator kernels

enum MMode {
  kApply = 0,      // y = M x
  kApplyDot = 1,   // y = M x, partial x.y
  kJacobi = 2,     // y = x + omega (b - M x) / D
  kJacobiDot = 3,  // y = x + omega (b - M x) / D, partial b.y
  kResid = 4,      // y = b - M x
  kDinvM = 5,      // y = (M x) / D, partial y.y
  kJacobi0 = 6,    // y = omega b / D   (first sweep from a zero guess)
  kDiag = 7,       // y = D
  kResidDot = 8,   // y = b - M x, partial y.y
  kJacobiZ = 9,    // two sweeps from a zero guess: y = x1 + omega (b - M x1) / D
                   // with x1 = omega b / D (x1 formed while staging; tiled
                   // kernel, constant viscosity only; x = b)
  kJacobiP = 10,   // sweep after the coarse-grid correction: y = x' + omega
                   // (b - M x') / D with x' = x + P e (prolongation of the
                   // coarse correction e added while staging; tiled kernel)
  kApplyDotP = 11  // CG direction update and product in one pass: p' = x + beta
                   // p (x = z, b = p, beta from the PCG state) formed while
                   // staging, y = M p', p' written to y2, partial p'.y
};

// Thread mapping: blockIdx.z = component * zchunks + z-chunk; each block
// covers kBlock consecutive (x fastest) faces of one z-plane of that
// component's array and loops over kz consecutive planes.
template <typename T, int DIM, bool VARMU, int MODE, int C>
__device__ __forceinline__ double face_op(const Op<T>& op, const T* __restrict__ x,
                                          const T* __restrict__ b, T* __restrict__ y, T omega,
                                          int idx, int k0, int kz) {
  const Grid& G = op.g;
  const int e0 = G.ext[C][0], e1 = G.ext[C][1], e2 = G.ext[C][2];
  double part = 0.0;
  if (idx >= e0 * e1) return part;
  const int j = idx / e0, i = idx - j * e0;
  const int ic_fixed = C == 0 ? i : (C == 1 ? j : -1);
  for (int k = k0; k < k0 + kz && k < e2; ++k) {
    const int ic = C == 2 ? k : ic_fixed;
    const int f = fidx<C>(G, i, j, k);
    if (!unk<C>(G, ic)) {
      y[f] = T(0);
      continue;
    }
    if (MODE == kJacobi0 || MODE == kDiag) {
      const T d = diag_M<T, DIM, VARMU, C>(op, i, j, k);
      y[f] = MODE == kDiag ? d : omega * b[f] / d;
      continue;
    }
    T mx, d;
    stencil_M<T, DIM, VARMU, C>(op, x, i, j, k, mx, d);
    T out;
    if (MODE == kApply || MODE == kApplyDot) {
      out = mx;
      if (MODE == kApplyDot) part += double(x[f]) * double(out);
    } else if (MODE == kJacobi || MODE == kJacobiDot) {
      const T bf = b[f];
      out = x[f] + omega * (bf - mx) / d;
      if (MODE == kJacobiDot) part += double(bf) * double(out);
    } else if (MODE == kResid || MODE == kResidDot) {
      out = b[f] - mx;
      if (MODE == kResidDot) part += double(out) * double(out);
    } else {  // kDinvM
      out = mx / d;
      part += double(out) * double(out);
    }
    y[f] = out;
  }
  return part;
}

template <typename T, int DIM, bool VARMU, int MODE>
__global__ __launch_bounds__(kBlock) void k_face_op(Op<T> op, const T* __restrict__ x,
                                                    const T* __restrict__ b, T* __restrict__ y,
                                                    T omega, int kz, int zchunks,
                                                    double* __restrict__ partial,
                                                    const PcgState* __restrict__ st) {
  if (st && st->done) return;
  const int c = blockIdx.z / zchunks;
  const int k0 = (blockIdx.z - c * zchunks) * kz;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  double part = 0.0;
  if (c == 0) part = face_op<T, DIM, VARMU, MODE, 0>(op, x, b, y, omega, idx, k0, kz);
  else if (c == 1) part = face_op<T, DIM, VARMU, MODE, 1>(op, x, b, y, omega, idx, k0, kz);
  else if (DIM == 3) part = face_op<T, DIM, VARMU, MODE, 2>(op, x, b, y, omega, idx, k0, kz);
  constexpr bool kRed = MODE == kApplyDot || MODE == kJacobiDot || MODE == kDinvM || MODE == kResidDot;
  if (kRed) {
    __shared__ double sh[kBlock / 64];
    double s = block_sum<kBlock>(part, sh);
    if (threadIdx.x == 0) partial[blockIdx.z * gridDim.x + blockIdx.x] = s;
  }
}

// out = s1 * (A q) + s2 * yv on unknown faces (yv may be null), 0 elsewhere
template <typename T, int C>
__device__ __forceinline__ void grad_face(const Grid& G, const T* __restrict__ q,
                                          const double* __restrict__ yv, double s1, double s2,
                                          double ih, double* __restrict__ out, int idx, int k0,
                                          int kz) {
  const int e0 = G.ext[C][0], e1 = G.ext[C][1], e2 = G.ext[C][2];
  if (idx >= e0 * e1) return;
  const int j = idx / e0, i = idx - j * e0;
  for (int k = k0; k < k0 + kz && k < e2; ++k) {
    const int ic = C == 0 ? i : (C == 1 ? j : k);
    const int f = fidx<C>(G, i, j, k);
    if (!unk<C>(G, ic)) {
      out[f] = 0.0;
      continue;
    }
    double v = s1 * double(grad_f<C>(G, q, i, j, k)) * ih;
    if (yv) v += s2 * yv[f];
    out[f] = v;
  }
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_grad_axpy(Grid G, const double* __restrict__ q,
                                                      const double* __restrict__ yv, double s1,
                                                      double s2, double* __restrict__ out, int kz,
                                                      int zchunks) {
  const int c = blockIdx.z / zchunks;
  const int k0 = (blockIdx.z - c * zchunks) * kz;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  const double ih = 1.0 / G.h;
  if (c == 0) grad_face<double, 0>(G, q, yv, s1, s2, ih, out, idx, k0, kz);
  else if (c == 1) grad_face<double, 1>(G, q, yv, s1, s2, ih, out, idx, k0, kz);
  else if (DIM == 3) grad_face<double, 2>(G, q, yv, s1, s2, ih, out, idx, k0, kz);
}

// t = s1 * (A^T x) + s2 * z on unpinned cells (z may be null), 0 at the pin;
// partial t.t and, if zz_partial, z.z over unpinned cells
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_div_axpy(Grid G, const T* __restrict__ x,
                                                     const T* __restrict__ z, double s1, double s2,
                                                     T* __restrict__ t, double* __restrict__ partial,
                                                     double* __restrict__ zz_partial) {
  const int nxy = G.n[0] * G.n[1];
  const int k = blockIdx.z;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  double a = 0.0, bz = 0.0;
  if (idx < nxy) {
    const int j = idx / G.n[0], i = idx - j * G.n[0];
    const int cc = cidx(G, i, j, k);
    double v = 0.0;
    if (cc != G.pin) {
      v = s1 * double(cdiv<DIM>(G, x, i, j, k)) / G.h;
      if (z) {
        const double zv = double(z[cc]);
        v += s2 * zv;
        bz = zv * zv;
      }
    }
    t[cc] = T(v);
    a = v * v;
  }
  __shared__ double sh[kBlock / 64];
  double s = block_sum<kBlock>(a, sh);
  if (threadIdx.x == 0 && partial) partial[blockIdx.z * gridDim.x + blockIdx.x] = s;
  if (zz_partial) {
    __syncthreads();
    double s2v = block_sum<kBlock>(bz, sh);
    if (threadIdx.x == 0) zz_partial[blockIdx.z * gridDim.x + blockIdx.x] = s2v;
  }
}

// FP64 velocity residual res = g - W w - A p on unknown faces; partials of
// res.res and g.g (unknown faces)
template <int DIM, bool VARMU, int C>
__device__ __forceinline__ void resid_face(const Op<double>& op, const double* __restrict__ g,
                                           const double* __restrict__ w,
                                           const double* __restrict__ p, double* __restrict__ res,
                                           int idx, int k0, int kz, double& rr, double& gg) {
  const Grid& G = op.g;
  const int e0 = G.ext[C][0], e1 = G.ext[C][1], e2 = G.ext[C][2];
  if (idx >= e0 * e1) return;
  const int j = idx / e0, i = idx - j * e0;
  for (int k = k0; k < k0 + kz && k < e2; ++k) {
    const int ic = C == 0 ? i : (C == 1 ? j : k);
    const int f = fidx<C>(G, i, j, k);
    if (!unk<C>(G, ic)) {
      if (res) res[f] = 0.0;
      continue;
    }
    double mx, d;
    stencil_M<double, DIM, VARMU, C>(op, w, i, j, k, mx, d);
    const double gf = g[f];
    const double v = gf - mx - grad_f<C>(G, p, i, j, k) * op.ih;
    if (res) res[f] = v;
    rr += v * v;
    gg += gf * gf;
  }
}

template <int DIM, bool VARMU>
__global__ __launch_bounds__(kBlock) void k_resid_w(Op<double> op, const double* __restrict__ g,
                                                    const double* __restrict__ w,
                                                    const double* __restrict__ p,
                                                    double* __restrict__ res, int kz, int zchunks,
                                                    double* __restrict__ part_rr,
                                                    double* __restrict__ part_gg) {
  const int c = blockIdx.z / zchunks;
  const int k0 = (blockIdx.z - c * zchunks) * kz;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  double rr = 0.0, gg = 0.0;
  if (c == 0) resid_face<DIM, VARMU, 0>(op, g, w, p, res, idx, k0, kz, rr, gg);
  else if (c == 1) resid_face<DIM, VARMU, 1>(op, g, w, p, res, idx, k0, kz, rr, gg);
  else if (DIM == 3) resid_face<DIM, VARMU, 2>(op, g, w, p, res, idx, k0, kz, rr, gg);
  __shared__ double sh[kBlock / 64];
  double s = block_sum<kBlock>(rr, sh);
  if (threadIdx.x == 0) part_rr[blockIdx.z * gridDim.x + blockIdx.x] = s;
  __syncthreads();
  s = block_sum<kBlock>(gg, sh);
  if (threadIdx.x == 0) part_gg[blockIdx.z * gridDim.x + blockIdx.x] = s;
}

// --------------------------------------------------------- vector kernels

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int n, T v, T* __restrict__ y) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = v;
}

// y = a x + b y
__global__ __launch_bounds__(kBlock) void k_axpby(int n, double a, const double* __restrict__ x,
                                                  double b, double* __restrict__ y) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    y[i] = a * x[i] + b * y[i];
}

// partial x.y
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot(int n, const T* __restrict__ x,
                                                const T* __restrict__ y, double* __restrict__ partial) {
  double s = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    s += double(x[i]) * double(y[i]);
  __shared__ double sh[kBlock / 64];
  s = block_sum<kBlock>(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_cast(int n, const TI* __restrict__ x, TO* __restrict__ y) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = TO(x[i]);
}

// GKB face update: v = s/alpha, Mv = y/alpha, u += zeta v
__global__ __launch_bounds__(kBlock) void k_gkb_faces(int n, double ialpha, double zeta,
                                                      const double* __restrict__ s,
                                                      const double* __restrict__ yv,
                                                      double* __restrict__ v, double* __restrict__ Mv,
                                                      double* __restrict__ u) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double vi = s[i] * ialpha;
    v[i] = vi;
    Mv[i] = yv[i] * ialpha;
    u[i] += zeta * vi;
  }
}

// GKB cell update: d = (q - beta d)/alpha, p -= zeta d
__global__ __launch_bounds__(kBlock) void k_gkb_cells(int n, double ialpha, double beta, double zeta,
                                                      const double* __restrict__ q,
                                                      double* __restrict__ d, double* __restrict__ p) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double di = (q[i] - beta * d[i]) * ialpha;
    d[i] = di;
    p[i] -= zeta * di;
  }
}

// --------------------------------------------------------------- PCG

// x = 0, r = f (cast), partial f.f
template <typename TI, typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_init(int n, const TI* __restrict__ f,
                                                     T* __restrict__ x, T* __restrict__ r,
                                                     double* __restrict__ part_ff) {
  double s = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const T fi = T(f[i]);
    x[i] = T(0);
    r[i] = fi;
    s += double(fi) * double(fi);
  }
  __shared__ double sh[kBlock / 64];
  s = block_sum<kBlock>(s, sh);
  if (threadIdx.x == 0) part_ff[blockIdx.x] = s;
}

// z = dinv r (Jacobi) when dinv != null; p = z; partial r.z
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_p0(int n, const T* __restrict__ dinv,
                                                   const T* __restrict__ r, T* __restrict__ z,
                                                   T* __restrict__ p, double* __restrict__ part_rz) {
  double s = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const T ri = r[i];
    const T zi = dinv ? dinv[i] * ri : z[i];
    if (dinv) z[i] = zi;
    p[i] = zi;
    s += double(ri) * double(zi);
  }
  __shared__ double sh[kBlock / 64];
  s = block_sum<kBlock>(s, sh);
  if (threadIdx.x == 0) part_rz[blockIdx.x] = s;
}

__global__ __launch_bounds__(kFinal) void k_pcg_start(PcgState* st, const double* part_ff, int nff,
                                                      const double* part_rz, int nrz, double tol,
                                                      int maxit) {
  __shared__ double sh[kFinal / 64];
  const double ff = sum_partials(part_ff, nff, sh);
  __syncthreads();
  const double rz = sum_partials(part_rz, nrz, sh);
  if (threadIdx.x == 0) {
    st->rr0 = ff;
    st->rr = ff;
    st->rz = rz;
    st->tol2 = tol * tol;
    st->it = 0;
    st->maxit = maxit;
    st->alpha = st->beta = st->pq = 0.0;
    st->rz_prev = rz;
    st->nonfinite = 0;
    st->done = (ff == 0.0) ? 1 : 0;
    st->status = 0;
    st->fallback = st->stagnant = st->use_zv = st->fallbacks = 0;
    st->fb_it = st->fb_reason = 0;
    st->theta = st->gain = st->gain_sum = 0.0;
    st->gain_n = 0;
    for (int i = 0; i < 10; ++i) st->ring[i] = 0.0;
  }
}

// Scalar steps of PCG on the device state (one thread): alpha from p.q;
// the convergence test on r.r (with rz: also beta, Jacobi path); beta from
// the new r.z.
__device__ __forceinline__ void pcg_set_alpha(PcgState* st, double pq) {
  st->pq = pq;
  const double a = st->rz / pq;
  if (!(pq > 0.0) || !isfinite(a)) {
    st->alpha = 0.0;
    st->nonfinite = 1;
    st->status = -4;
    st->done = 1;
  } else {
    st->alpha = a;
  }
}
__device__ __forceinline__ void pcg_set_check(PcgState* st, double rr, bool has_rz, double rz) {
  st->rr = rr;
  st->it += 1;
  // r.r sampled every 5 iterations: stagnant when no decrease over 50
  // (CG minimises the energy norm, so r.r may rise over shorter spans)
  if (st->it % 5 == 0) {
    const int slot = (st->it / 5) % 10;
    if (st->it > 50 && rr >= st->ring[slot]) st->stagnant = 1;
    st->ring[slot] = rr;
  }
  if (!isfinite(rr)) {
    st->nonfinite = 1;
    st->status = -4;
    st->done = 1;
  } else if (rr <= st->tol2 * st->rr0) {
    st->done = 1;
    st->status = 0;
  } else if (st->it >= st->maxit) {
    st->done = 1;
    st->status = -5;
  } else if (has_rz) {
    st->beta = rz / st->rz;
    st->rz = rz;
  }
}
__device__ __forceinline__ void pcg_set_beta(PcgState* st, double rz) {
  st->beta = rz / st->rz;
  st->rz = rz;
}

// The one-block scalar kernels below read the done flag together with the
// partials (the flag is tested once both loads are in flight).
__global__ __launch_bounds__(kFinal) void k_pcg_alpha(PcgState* st, const double* part_pq, int n) {
  const int done = st->done;
  const double v = thread_partials(part_pq, n);
  if (done) return;
  __shared__ double sh[kFinal / 64];
  const double pq = block_sum<kFinal>(v, sh);
  if (threadIdx.x == 0) pcg_set_alpha(st, pq);
}

// x += alpha p, r -= alpha q; partial r.r; Jacobi (dinv != null): z = dinv r
// and partial r.z
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_xr(int n, const PcgState* __restrict__ st,
                                                   const T* __restrict__ p, const T* __restrict__ q,
                                                   T* __restrict__ x, T* __restrict__ r,
                                                   const T* __restrict__ dinv, T* __restrict__ z,
                                                   double* __restrict__ part_rr,
                                                   double* __restrict__ part_rz) {
  // the flag and alpha are tested / used once this thread's first loads are
  // in flight
  const int done = st->done;
  const T a = T(st->alpha);
  double s = 0.0, t = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const T xi = x[i], pi = p[i], r0 = r[i], qi = q[i];
    if (done) break;
    x[i] = xi + a * pi;
    const T ri = r0 - a * qi;
    r[i] = ri;
    s += double(ri) * double(ri);
    if (dinv) {
      const T zi = dinv[i] * ri;
      z[i] = zi;
      t += double(ri) * double(zi);
    }
  }
  if (done) return;  // uniform: every thread of the block leaves
  __shared__ double sh[kBlock / 64];
  double v = block_sum<kBlock>(s, sh);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = v;
  if (dinv) {
    __syncthreads();
    v = block_sum<kBlock>(t, sh);
    if (threadIdx.x == 0) part_rz[blockIdx.x] = v;
  }
}

// convergence test on r.r; with part_rz also the CG beta (Jacobi path)
__global__ __launch_bounds__(kFinal) void k_pcg_check(PcgState* st, const double* part_rr, int nrr,
                                                      const double* part_rz, int nrz) {
  const int done = st->done;
  const double vrr = thread_partials(part_rr, nrr);
  const double vrz = part_rz ? thread_partials(part_rz, nrz) : 0.0;
  if (done) return;
  __shared__ double sh[kFinal / 64];
  const double rr = block_sum<kFinal>(vrr, sh);
  double rz = 0.0;
  if (part_rz) {
    __syncthreads();
    rz = block_sum<kFinal>(vrz, sh);
  }
  if (threadIdx.x == 0) pcg_set_check(st, rr, part_rz != nullptr, rz);
}

// preconditioned path: rz_new from the partials of the last V-cycle kernel
__global__ __launch_bounds__(kFinal) void k_pcg_beta(PcgState* st, const double* part_rz, int n) {
  const int done = st->done;
  const double v = thread_partials(part_rz, n);
  if (done) return;
  __shared__ double sh[kFinal / 64];
  const double rz = block_sum<kFinal>(v, sh);
  if (threadIdx.x == 0) pcg_set_beta(st, rz);
}

// p = z + beta p
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_p(int n, const PcgState* __restrict__ st,
                                                  const T* __restrict__ z, T* __restrict__ p) {
  if (st->done) return;
  const T b = T(st->beta);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    p[i] = z[i] + b * p[i];
}

// ------------------------------------------------------------ multigrid

// Tangential weights of the two transfer pairs.  DIV (divergence
// compatible): a fine face takes the value of the coarse face whose cell
// pair covers it, constant across the two fine cells in each tangential
// direction.  SMOOTH: linear in each tangential direction between the
// centres of the coarse rows, 3/4 from the row that covers the fine row and
// 1/4 from the next row on the fine row's side; beyond a side that next row
// is a mirror ghost, -1 times the covering row at a DIRICHLET wall (zero
// tangential velocity on the wall) and +1 times it at a NATURAL side.
// Weight of coarse row T in the value of fine row t along a tangential axis
// with nc coarse rows and side types lo / hi:
__device__ __forceinline__ double tan_weight(int t, int T, int nc, int lo, int hi) {
  const int Tc = t >> 1, Tn = (t & 1) ? Tc + 1 : Tc - 1;
  double w = 0.0;
  if (Tc == T) {
    w = 0.75;
    if (Tn < 0) w += lo == kDir ? -0.25 : 0.25;
    if (Tn >= nc) w += hi == kDir ? -0.25 : 0.25;
  } else if (Tn == T) {
    w = 0.25;
  }
  return w;
}

// Restriction of face residuals, full weighting: coarse face = (1/2^d) *
// sum over the fine faces it covers, normal neighbours weighted 1/2
// (transpose of the prolongation below divided by 2^d); SMOOTH also takes
// the fine rows next to the covered ones in each tangential direction, with
// the transposed weights.
// x0c (optional): the coarse level's first smoothing sweep from a zero
// guess, x0c = omega_c dinv_c bc, written in the same pass
template <typename T>
struct Pair2;
template <>
struct Pair2<float> {
  typedef float2 type;
};
template <>
struct Pair2<double> {
  typedef double2 type;
};

// pair: the fine v and w faces 2i, 2i+1 of a row sit at an even (aligned)
// index (x extent and array offsets even), so the DIV transfer in 3D loads
// them as one pair (they share the mask of their normal index); the sum
// keeps the order of the general loop below, so both give the same bits
template <typename T, int DIM, int C, bool SM>
__device__ __forceinline__ void restrict_face(const Grid& Gf, const Grid& Gc,
                                              const T* __restrict__ rf, T* __restrict__ bc,
                                              const T* __restrict__ dinv_c, T omega_c,
                                              T* __restrict__ x0c, int idx, int k, int done,
                                              int pair) {
  const int e0 = Gc.ext[C][0], e1 = Gc.ext[C][1];
  if (idx >= e0 * e1 || k >= Gc.ext[C][2]) return;
  const int j = idx / e0, i = idx - j * e0;
  const int P[3] = {i, j, k};
  const int f = fidx<C>(Gc, i, j, k);
  if (!unk<C>(Gc, P[C])) {
    if (done) return;
    bc[f] = T(0);
    if (x0c) x0c[f] = T(0);
    return;
  }
  T acc = T(0);
  const int nfC = Gf.n[C];
  const int A1 = (C + 1) % DIM;
  const int A2 = (C + 2) % 3;
  // fine rows per tangential axis: the two covered ones (DIV), with one
  // more on each side (SMOOTH)
  constexpr int kT = SM ? 4 : 2, kT0 = SM ? -1 : 0;
  if constexpr (!SM && DIM == 3 && C != 0) {
    if (pair) {  // uniform
      // x is a tangential axis; B the other one (z for v, y for w).  The
      // general loop runs (dn, A1, A2): for v A1 = z, A2 = x, for w A1 = x,
      // A2 = y
      constexpr int B = C == 1 ? 2 : 1;
      typedef typename Pair2<T>::type T2;
#pragma unroll
      for (int dn = -1; dn <= 1; ++dn) {
        const int fn = 2 * P[C] + dn;
        if (fn < 0 || fn > nfC) continue;
        const T wn = dn == 0 ? T(1) : T(0.5);
        const bool on = unk<C>(Gf, fn);
        T2 pb[2];
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
          int Q[3];
          Q[C] = fn;
          Q[0] = 2 * P[0];
          Q[B] = 2 * P[B] + tb;
          pb[tb] = on ? *reinterpret_cast<const T2*>(rf + fidx<C>(Gf, Q[0], Q[1], Q[2]))
                      : T2{T(0), T(0)};
        }
        if (C == 1) {  // (z, x) order
          acc += wn * pb[0].x;
          acc += wn * pb[0].y;
          acc += wn * pb[1].x;
          acc += wn * pb[1].y;
        } else {  // (x, y) order
          acc += wn * pb[0].x;
          acc += wn * pb[1].x;
          acc += wn * pb[0].y;
          acc += wn * pb[1].y;
        }
      }
      const T dc = x0c ? dinv_c[f] : T(0);
      if (done) return;
      const T v = acc * T(0.125);
      bc[f] = v;
      if (x0c) x0c[f] = omega_c * dc * v;
      return;
    }
  }
#pragma unroll
  for (int dn = -1; dn <= 1; ++dn) {
    const int fn = 2 * P[C] + dn;
    if (fn < 0 || fn > nfC) continue;
    const T wn = dn == 0 ? T(1) : T(0.5);
#pragma unroll
    for (int t1 = 0; t1 < kT; ++t1)
#pragma unroll
      for (int t2 = 0; t2 < (DIM == 3 ? kT : 1); ++t2) {
        int Q[3];
        Q[C] = fn;
        Q[A1] = 2 * P[A1] + kT0 + t1;
        if (DIM == 3) Q[A2] = 2 * P[A2] + kT0 + t2;
        else Q[2] = 0;
        T w = wn;
        if (SM) {
          if (Q[A1] < 0 || Q[A1] >= Gf.n[A1]) continue;
          w *= T(tan_weight(Q[A1], P[A1], Gc.n[A1], Gc.bc[2 * A1], Gc.bc[2 * A1 + 1]));
          if (DIM == 3) {
            if (Q[A2] < 0 || Q[A2] >= Gf.n[A2]) continue;
            w *= T(tan_weight(Q[A2], P[A2], Gc.n[A2], Gc.bc[2 * A2], Gc.bc[2 * A2 + 1]));
          }
        }
        acc += w * ldm<C>(Gf, rf, Q[0], Q[1], Q[2]);
      }
  }
  const T dc = x0c ? dinv_c[f] : T(0);
  if (done) return;
  const T v = acc * T(DIM == 3 ? 0.125 : 0.25);
  bc[f] = v;
  if (x0c) x0c[f] = omega_c * dc * v;
}

template <typename T, int DIM, bool SM>
__global__ __launch_bounds__(kBlock) void k_restrict(Grid Gf, Grid Gc, const T* __restrict__ rf,
                                                     T* __restrict__ bc, const PcgState* st,
                                                     const T* __restrict__ dinv_c = nullptr,
                                                     T omega_c = T(0), T* __restrict__ x0c = nullptr,
                                                     int pair = 0) {
  // the flag is tested after the fine values are loaded
  const int done = st ? st->done : 0;
  const int c = blockIdx.z / Gc.nze;
  const int k = blockIdx.z - c * Gc.nze;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (c == 0) restrict_face<T, DIM, 0, SM>(Gf, Gc, rf, bc, dinv_c, omega_c, x0c, idx, k, done, pair);
  else if (c == 1) restrict_face<T, DIM, 1, SM>(Gf, Gc, rf, bc, dinv_c, omega_c, x0c, idx, k, done, pair);
  else if (DIM == 3) restrict_face<T, DIM, 2, SM>(Gf, Gc, rf, bc, dinv_c, omega_c, x0c, idx, k, done, pair);
}

// Prolongation + correction: fine faces coinciding with a coarse face take
// its value, fine faces between two coarse faces the mean (linear in the
// normal direction); across the two fine cells in tangential directions
// constant (DIV) or linear between coarse row centres (SMOOTH, weights of
// tan_weight).
template <typename T, int DIM, int C, bool SM>
__device__ __forceinline__ void prolong_face(const Grid& Gf, const Grid& Gc,
                                             const T* __restrict__ ec, T* __restrict__ xf, int idx,
                                             int k) {
  const int e0 = Gf.ext[C][0], e1 = Gf.ext[C][1];
  if (idx >= e0 * e1 || k >= Gf.ext[C][2]) return;
  const int j = idx / e0, i = idx - j * e0;
  const int P[3] = {i, j, k};
  if (!unk<C>(Gf, P[C])) return;
  int Q[3] = {P[0] >> 1, P[1] >> 1, P[2] >> 1};
  Q[C] = P[C] >> 1;
  T v;
  if (!SM) {
    v = ldm<C>(Gc, ec, Q[0], Q[1], Q[2]);
    if (P[C] & 1) {
      int R[3] = {Q[0], Q[1], Q[2]};
      R[C] += 1;
      v = T(0.5) * (v + ldm<C>(Gc, ec, R[0], R[1], R[2]));
    }
  } else {
    const int A1 = (C + 1) % DIM, A2 = (C + 2) % 3;
    const bool odd = P[C] & 1;
    v = T(0);
#pragma unroll
    for (int dn = 0; dn < 2; ++dn) {
      if (dn == 1 && !odd) break;
      const T wn = odd ? T(0.5) : T(1);
#pragma unroll
      for (int a1 = 0; a1 < 2; ++a1) {
        int R[3] = {Q[0], Q[1], Q[2]};
        R[C] += dn;
        if (a1 == 1) R[A1] += (P[A1] & 1) ? 1 : -1;
        if (R[A1] < 0 || R[A1] >= Gc.n[A1]) continue;  // folded into a1 = 0
        const T w1 = T(tan_weight(P[A1], R[A1], Gc.n[A1], Gc.bc[2 * A1], Gc.bc[2 * A1 + 1]));
#pragma unroll
        for (int a2 = 0; a2 < (DIM == 3 ? 2 : 1); ++a2) {
          if (DIM == 3) {
            R[A2] = Q[A2] + (a2 == 1 ? ((P[A2] & 1) ? 1 : -1) : 0);
            if (R[A2] < 0 || R[A2] >= Gc.n[A2]) continue;
          }
          const T w2 = DIM == 3 ? T(tan_weight(P[A2], R[A2], Gc.n[A2], Gc.bc[2 * A2],
                                               Gc.bc[2 * A2 + 1]))
                                : T(1);
          v += wn * w1 * w2 * ldm<C>(Gc, ec, R[0], R[1], R[2]);
        }
      }
    }
  }
  xf[fidx<C>(Gf, i, j, k)] += v;
}

template <typename T, int DIM, bool SM>
__global__ __launch_bounds__(kBlock) void k_prolong_add(Grid Gf, Grid Gc, const T* __restrict__ ec,
                                                        T* __restrict__ xf, const PcgState* st) {
  if (st && st->done) return;
  const int c = blockIdx.z / Gf.nze;
  const int k = blockIdx.z - c * Gf.nze;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (c == 0) prolong_face<T, DIM, 0, SM>(Gf, Gc, ec, xf, idx, k);
  else if (c == 1) prolong_face<T, DIM, 1, SM>(Gf, Gc, ec, xf, idx, k);
  else if (DIM == 3) prolong_face<T, DIM, 2, SM>(Gf, Gc, ec, xf, idx, k);
}

// x = Minv b on the coarsest grid: FP64 dense inverse (full-face layout,
// zero rows/columns at non-unknown faces); one wave64 per row, b staged in LDS
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_gemv(int m, const double* __restrict__ Minv,
                                                        const T* __restrict__ b, T* __restrict__ x,
                                                        const PcgState* st) {
  const int done = st ? st->done : 0;
  extern __shared__ __align__(16) double sb[];
  for (int i = threadIdx.x; i < m; i += kBlock) sb[i] = double(b[i]);
  if (done) return;  // uniform, before the barrier
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (row >= m) return;
  const double* a = Minv + (size_t)row * m;
  double s = 0.0;
  if ((m & 1) == 0) {
    // 16-byte loads, four independent partial sums: more loads in flight
    const double2* a2 = reinterpret_cast<const double2*>(a);
    const double2* b2 = reinterpret_cast<const double2*>(sb);
    const int h = m >> 1;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int c = lane;
    for (; c + 64 < h; c += 128) {
      const double2 u = a2[c], v = a2[c + 64], bu = b2[c], bv = b2[c + 64];
      s0 += u.x * bu.x;
      s1 += u.y * bu.y;
      s2 += v.x * bv.x;
      s3 += v.y * bv.y;
    }
    for (; c < h; c += 64) {
      const double2 u = a2[c], bu = b2[c];
      s0 += u.x * bu.x;
      s1 += u.y * bu.y;
    }
    s = (s0 + s1) + (s2 + s3);
  } else {
    for (int c = lane; c < m; c += 64) s += a[c] * sb[c];
  }
  s = wave_sum(s);
  if (lane == 0) x[row] = T(s);
}

}  // namespace gkb
