// Assembled (CSR) saddle systems: the operators of the GKB iteration for a
// user's W (m x m) and A (m x n) given as compressed sparse rows, as a PETSc
// fieldsplit user passes them (Section 3), with the optional central block
// scaling blockdiag(D^-1/2, R^-1/2) of Section 4.1, D = diag(W),
// R = diag(A^T D^-1 A).  The scaling is applied on the fly: with
// s_w = D^-1/2 and s_p = R^-1/2 the scaled operators are
//   W' x = s_w .* (W (s_w .* x)),  A' p = s_w .* (A (s_p .* p)),
//   A'^T x = s_p .* (A^T (s_w .* x)),
// so the unscaled system stays available for the residual.  One thread per
// row (the rows of FD / FEM Stokes blocks hold a few to a few dozen
// entries); A^T is a transposed copy built at setup so that every product is
// a row gather without atomics, and every reduction is deterministic (block
// partials, fixed order).
#pragma once
#include "kernels.hpp"

namespace gkb {

template <typename T>
struct CsrMat {
  int rows = 0;
  const int* ptr = nullptr;  // rows + 1
  const int* col = nullptr;
  const T* val = nullptr;
};

template <typename T>
struct CsrOps {
  CsrMat<T> W, A, AT;      // AT: n x m
  const T* sw = nullptr;   // D^-1/2 (null: no scaling)
  const T* sp = nullptr;   // R^-1/2
  int m = 0, n = 0;
};

template <typename T>
__device__ __forceinline__ T sget(const T* s, int i) {
  return s ? s[i] : T(1);
}

// row i of the (scaled) product M x = W' x + eta A' t with t = A'^T x given
template <typename T>
__device__ __forceinline__ T csr_M_row(const CsrOps<T>& o, T eta, const T* __restrict__ x,
                                       const T* __restrict__ t, int i, T* diag) {
  const T si = sget(o.sw, i);
  T acc = T(0), d = T(0);
  for (int e = o.W.ptr[i]; e < o.W.ptr[i + 1]; ++e) {
    const int j = o.W.col[e];
    const T a = o.W.val[e];
    acc += a * (sget(o.sw, j) * x[j]);
    if (j == i) d += a * si * si;
  }
  acc *= si;
  if (eta != T(0)) {
    T ga = T(0), dd = T(0);
    for (int e = o.A.ptr[i]; e < o.A.ptr[i + 1]; ++e) {
      const int k = o.A.col[e];
      const T a = o.A.val[e] * sget(o.sp, k);
      if (t) ga += a * t[k];
      dd += a * a;
    }
    acc += eta * si * ga;
    d += eta * si * si * dd;
  }
  if (diag) *diag = d;
  return acc;
}

// t = A'^T x (pressure-shaped)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_at(CsrOps<T> o, const T* __restrict__ x,
                                                   T* __restrict__ t,
                                                   const PcgState* __restrict__ st) {
  if (st && st->done) return;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < o.n; k += gridDim.x * kBlock) {
    T acc = T(0);
    for (int e = o.AT.ptr[k]; e < o.AT.ptr[k + 1]; ++e) {
      const int i = o.AT.col[e];
      acc += o.AT.val[e] * (sget(o.sw, i) * x[i]);
    }
    t[k] = sget(o.sp, k) * acc;
  }
}

// M-apply modes of the face-operator family (kApply, kApplyDot, kResid,
// kResidDot, kDiag), with t = A'^T x from k_csr_at (unused for eta = 0 and
// for kDiag)
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_csr_m(CsrOps<T> o, T eta, const T* __restrict__ x,
                                                  const T* __restrict__ t,
                                                  const T* __restrict__ b, T* __restrict__ y,
                                                  double* __restrict__ partial,
                                                  const PcgState* __restrict__ st) {
  if (st && st->done) return;
  double part = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < o.m; i += gridDim.x * kBlock) {
    T d = T(0);
    if (MODE == kDiag) {
      csr_M_row<T>(o, eta, x, nullptr, i, &d);
      y[i] = d;
      continue;
    }
    const T mx = csr_M_row<T>(o, eta, x, t, i, nullptr);
    T out;
    if (MODE == kApply || MODE == kApplyDot) {
      out = mx;
      if (MODE == kApplyDot) part += double(x[i]) * double(out);
    } else {  // kResid, kResidDot
      out = b[i] - mx;
      if (MODE == kResidDot) part += double(out) * double(out);
    }
    y[i] = out;
  }
  if (MODE == kApplyDot || MODE == kResidDot) {
    __shared__ double sh[kBlock / 64];
    const double s = block_sum<kBlock>(part, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// out = s1 (A' q) + s2 yv (yv may be null), FP64
__global__ __launch_bounds__(kBlock) void k_csr_grad(CsrOps<double> o, const double* __restrict__ q,
                                                     const double* __restrict__ yv, double s1,
                                                     double s2, double* __restrict__ out) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < o.m; i += gridDim.x * kBlock) {
    double acc = 0.0;
    for (int e = o.A.ptr[i]; e < o.A.ptr[i + 1]; ++e) {
      const int k = o.A.col[e];
      acc += o.A.val[e] * (sget(o.sp, k) * q[k]);
    }
    double v = s1 * sget(o.sw, i) * acc;
    if (yv) v += s2 * yv[i];
    out[i] = v;
  }
}

// t = s1 (A'^T x) + s2 z (z may be null); partials of t.t and, with
// zz_partial, z.z
template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_div(CsrOps<T> o, const T* __restrict__ x,
                                                    const T* __restrict__ z, double s1, double s2,
                                                    T* __restrict__ t, double* __restrict__ partial,
                                                    double* __restrict__ zz_partial) {
  double a = 0.0, bz = 0.0;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < o.n; k += gridDim.x * kBlock) {
    double acc = 0.0;
    for (int e = o.AT.ptr[k]; e < o.AT.ptr[k + 1]; ++e) {
      const int i = o.AT.col[e];
      acc += double(o.AT.val[e]) * (double(sget(o.sw, i)) * double(x[i]));
    }
    double v = s1 * double(sget(o.sp, k)) * acc;
    if (z) {
      const double zv = double(z[k]);
      v += s2 * zv;
      bz += zv * zv;
    }
    t[k] = T(v);
    a += v * v;
  }
  __shared__ double sh[kBlock / 64];
  const double s = block_sum<kBlock>(a, sh);
  if (threadIdx.x == 0 && partial) partial[blockIdx.x] = s;
  if (zz_partial) {
    __syncthreads();
    const double s2v = block_sum<kBlock>(bz, sh);
    if (threadIdx.x == 0) zz_partial[blockIdx.x] = s2v;
  }
}

// FP64 velocity residual res = g - W' w - A' p; partials of res.res and g.g
__global__ __launch_bounds__(kBlock) void k_csr_resid_w(CsrOps<double> o,
                                                        const double* __restrict__ g,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ p,
                                                        double* __restrict__ res,
                                                        double* __restrict__ part_rr,
                                                        double* __restrict__ part_gg) {
  double rr = 0.0, gg = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < o.m; i += gridDim.x * kBlock) {
    const double si = sget(o.sw, i);
    double wx = 0.0, ap = 0.0;
    for (int e = o.W.ptr[i]; e < o.W.ptr[i + 1]; ++e) {
      const int j = o.W.col[e];
      wx += o.W.val[e] * (sget(o.sw, j) * w[j]);
    }
    for (int e = o.A.ptr[i]; e < o.A.ptr[i + 1]; ++e) {
      const int k = o.A.col[e];
      ap += o.A.val[e] * (sget(o.sp, k) * p[k]);
    }
    const double gi = g[i];
    const double v = gi - si * wx - si * ap;
    if (res) res[i] = v;
    rr += v * v;
    gg += gi * gi;
  }
  __shared__ double sh[kBlock / 64];
  double s = block_sum<kBlock>(rr, sh);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
  __syncthreads();
  s = block_sum<kBlock>(gg, sh);
  if (threadIdx.x == 0) part_gg[blockIdx.x] = s;
}

// y = s .* x (scaling of right-hand sides and solutions)
__global__ __launch_bounds__(kBlock) void k_scale(int n, const double* __restrict__ s,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ y) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = s[i] * x[i];
}

}  // namespace gkb
