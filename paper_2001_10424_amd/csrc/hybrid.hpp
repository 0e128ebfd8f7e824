// Edge-space (vector potential) smoothing for M = W + eta A A^T.
//
// Point-Jacobi on M cannot damp the oscillatory divergence-free error of a
// level once eta >> mu: those fields see only W, a thousandth of the diagonal
// that scales the sweep.  Every discretely divergence-free face field of the
// MAC grid is a discrete curl C psi of an edge field psi (a stream function
// on the vertices in 2D), and A^T C = 0, so M C = W C.  The hybrid smoother
// follows each weighted-Jacobi sweep on M by a weighted-Jacobi sweep on the
// edge operator C^T W C,
//     x += C omega_e D_e^-1 C^T (b - M x),   D_e = diag(C^T W C),
// which acts on exactly the fields the face sweep misses (Hiptmair's hybrid
// smoother for H(div) problems, here with Jacobi in both spaces).  Applied
// as (face, edge) before and (edge, face) after the coarse correction, the
// V-cycle stays symmetric.
//
// Edge storage: the point grid of the cells, component-major.  3D point
// (i, j, k) carries the x-edge (i+1/2, j, k), the y-edge (i, j+1/2, k) and
// the z-edge (i, j, k+1/2), i.e. the edges through the lowest corner of cell
// (i, j, k); 2D point (i, j) carries the vertex (i, j).  Edges beyond the
// point grid are 0, and so is every edge lying in a DIRICHLET wall, which
// keeps C psi zero on the faces that are not unknowns.  With these
// conventions
//     u(p) = psi_z(p + e_y) - psi_z(p) - psi_y(p + e_z) + psi_y(p)
//     v(p) = psi_x(p + e_z) - psi_x(p) - psi_z(p + e_x) + psi_z(p)
//     w(p) = psi_y(p + e_x) - psi_y(p) - psi_x(p + e_y) + psi_x(p)
// (2D: u(p) = psi(p + e_y) - psi(p), v(p) = psi(p) - psi(p + e_x)) on the
// lower faces of cell p, and C^T is the exact transpose.  The 1/h of the
// curl is left out: D_e absorbs the scale.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace gkb {

template <int DIM>
constexpr int edge_comps() { return DIM == 3 ? 3 : 1; }

// edge component a at point (i, j, k) lies in a DIRICHLET wall
template <int DIM>
__device__ __forceinline__ bool edge_in_wall(const Grid& G, int a, int i, int j, int k) {
  const bool wx = i == 0 && G.bc[0] == kDir;
  const bool wy = j == 0 && G.bc[2] == kDir;
  const bool wz = DIM == 3 && k == 0 && G.bc[4] == kDir;
  if (DIM == 2) return wx || wy;
  if (a == 0) return wy || wz;  // x-edge: planes y = j and z = k
  if (a == 1) return wx || wz;
  return wx || wy;
}

// value of face component C at point (i, j, k) of the lower-face lattice;
// 0 outside the point grid
template <int C, typename T>
__device__ __forceinline__ T face_at(const Grid& G, const T* __restrict__ r, int i, int j, int k) {
  if (i < 0 || j < 0 || k < 0) return T(0);
  return r[fidx<C>(G, i, j, k)];
}

// psi = omega dinv (C^T r) on every edge (dinv == nullptr: unscaled C^T r);
// edges in a DIRICHLET wall get 0.  Grid: cell planes (x fastest).
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_edge_ct(Grid G, const T* __restrict__ r,
                                                    const T* __restrict__ dinv, T omega,
                                                    T* __restrict__ psi, const PcgState* st) {
  if (st && st->done) return;
  const int k = blockIdx.z;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= G.n[0] * G.n[1]) return;
  const int j = idx / G.n[0], i = idx - j * G.n[0];
  const long nc = G.n_cells;
  const long p = (long)k * G.n[0] * G.n[1] + idx;
  if (DIM == 2) {
    T t = face_at<0>(G, r, i, j - 1, 0) - face_at<0>(G, r, i, j, 0) -
          face_at<1>(G, r, i - 1, j, 0) + face_at<1>(G, r, i, j, 0);
    if (edge_in_wall<2>(G, 0, i, j, 0)) t = T(0);
    else t *= dinv ? omega * dinv[p] : omega;
    psi[p] = t;
    return;
  }
  const T du = face_at<0>(G, r, i, j, k), dv = face_at<1>(G, r, i, j, k),
          dw = face_at<2>(G, r, i, j, k);
  T tx = face_at<1>(G, r, i, j, k - 1) - dv - face_at<2>(G, r, i, j - 1, k) + dw;
  T ty = du - face_at<0>(G, r, i, j, k - 1) + face_at<2>(G, r, i - 1, j, k) - dw;
  T tz = face_at<0>(G, r, i, j - 1, k) - du - face_at<1>(G, r, i - 1, j, k) + dv;
  tx = edge_in_wall<3>(G, 0, i, j, k) ? T(0) : tx * (dinv ? omega * dinv[p] : omega);
  ty = edge_in_wall<3>(G, 1, i, j, k) ? T(0) : ty * (dinv ? omega * dinv[nc + p] : omega);
  tz = edge_in_wall<3>(G, 2, i, j, k) ? T(0) : tz * (dinv ? omega * dinv[2 * nc + p] : omega);
  psi[p] = tx;
  psi[nc + p] = ty;
  psi[2 * nc + p] = tz;
}

template <typename T>
__device__ __forceinline__ T pt(const Grid& G, const T* __restrict__ a, int i, int j, int k) {
  if (i >= G.n[0] || j >= G.n[1] || k >= G.n[2]) return T(0);
  return a[((long)k * G.n[1] + j) * G.n[0] + i];
}

// x += C psi on the unknown faces (the lower faces of each cell; C psi is 0
// on the upper boundary faces)
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_curl_add(Grid G, const T* __restrict__ psi,
                                                     T* __restrict__ x, const PcgState* st) {
  if (st && st->done) return;
  const int k = blockIdx.z;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= G.n[0] * G.n[1]) return;
  const int j = idx / G.n[0], i = idx - j * G.n[0];
  const long nc = G.n_cells;
  if (DIM == 2) {
    const T s = pt(G, psi, i, j, 0);
    if (unk<0>(G, i)) x[fidx<0>(G, i, j, 0)] += pt(G, psi, i, j + 1, 0) - s;
    if (unk<1>(G, j)) x[fidx<1>(G, i, j, 0)] += s - pt(G, psi, i + 1, j, 0);
    return;
  }
  const T* px = psi;
  const T* py = psi + nc;
  const T* pz = psi + 2 * nc;
  const T sx = pt(G, px, i, j, k), sy = pt(G, py, i, j, k), sz = pt(G, pz, i, j, k);
  if (unk<0>(G, i))
    x[fidx<0>(G, i, j, k)] += pt(G, pz, i, j + 1, k) - sz - pt(G, py, i, j, k + 1) + sy;
  if (unk<1>(G, j))
    x[fidx<1>(G, i, j, k)] += pt(G, px, i, j, k + 1) - sx - pt(G, pz, i + 1, j, k) + sz;
  if (unk<2>(G, k))
    x[fidx<2>(G, i, j, k)] += pt(G, py, i + 1, j, k) - sy - pt(G, px, i, j + 1, k) + sx;
}

// psi_A = omega dinv_A (C^T r)_A at point (i, j, k) >= 0; 0 beyond the point
// grid or in a DIRICHLET wall
template <typename T, int DIM, int A>
__device__ __forceinline__ T edge_psi(const Grid& G, const T* __restrict__ r,
                                      const T* __restrict__ dinv, T omega, int i, int j, int k) {
  if (i >= G.n[0] || j >= G.n[1] || k >= G.n[2] || edge_in_wall<DIM>(G, A, i, j, k)) return T(0);
  T t;
  if (DIM == 2)
    t = face_at<0>(G, r, i, j - 1, 0) - face_at<0>(G, r, i, j, 0) - face_at<1>(G, r, i - 1, j, 0) +
        face_at<1>(G, r, i, j, 0);
  else if (A == 0)
    t = face_at<1>(G, r, i, j, k - 1) - face_at<1>(G, r, i, j, k) - face_at<2>(G, r, i, j - 1, k) +
        face_at<2>(G, r, i, j, k);
  else if (A == 1)
    t = face_at<0>(G, r, i, j, k) - face_at<0>(G, r, i, j, k - 1) + face_at<2>(G, r, i - 1, j, k) -
        face_at<2>(G, r, i, j, k);
  else
    t = face_at<0>(G, r, i, j - 1, k) - face_at<0>(G, r, i, j, k) - face_at<1>(G, r, i - 1, j, k) +
        face_at<1>(G, r, i, j, k);
  const long p = ((long)k * G.n[1] + j) * G.n[0] + i;
  return omega * dinv[(long)A * G.n_cells + p] * t;
}

// The edge half of the hybrid smoother in one pass: x += C omega D_e^-1 C^T r
// on the lower faces of every cell.  Each point evaluates the edge values its
// three faces need (nine in 3D, three in 2D) straight from r; neighbouring
// points share those reads through the caches, and the edge field is never
// stored.
template <typename T, int DIM>
__global__ __launch_bounds__(kBlock) void k_edge_smooth(Grid G, const T* __restrict__ r,
                                                        const T* __restrict__ dinv, T omega,
                                                        T* __restrict__ x, const PcgState* st) {
  if (st && st->done) return;
  const int k = blockIdx.z;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= G.n[0] * G.n[1]) return;
  const int j = idx / G.n[0], i = idx - j * G.n[0];
  if (DIM == 2) {
    const T s = edge_psi<T, 2, 0>(G, r, dinv, omega, i, j, 0);
    if (unk<0>(G, i)) x[fidx<0>(G, i, j, 0)] += edge_psi<T, 2, 0>(G, r, dinv, omega, i, j + 1, 0) - s;
    if (unk<1>(G, j)) x[fidx<1>(G, i, j, 0)] += s - edge_psi<T, 2, 0>(G, r, dinv, omega, i + 1, j, 0);
    return;
  }
  const T sx = edge_psi<T, 3, 0>(G, r, dinv, omega, i, j, k);
  const T sy = edge_psi<T, 3, 1>(G, r, dinv, omega, i, j, k);
  const T sz = edge_psi<T, 3, 2>(G, r, dinv, omega, i, j, k);
  if (unk<0>(G, i))
    x[fidx<0>(G, i, j, k)] += edge_psi<T, 3, 2>(G, r, dinv, omega, i, j + 1, k) - sz -
                              edge_psi<T, 3, 1>(G, r, dinv, omega, i, j, k + 1) + sy;
  if (unk<1>(G, j))
    x[fidx<1>(G, i, j, k)] += edge_psi<T, 3, 0>(G, r, dinv, omega, i, j, k + 1) - sx -
                              edge_psi<T, 3, 2>(G, r, dinv, omega, i + 1, j, k) + sz;
  if (unk<2>(G, k))
    x[fidx<2>(G, i, j, k)] += edge_psi<T, 3, 1>(G, r, dinv, omega, i + 1, j, k) - sy -
                              edge_psi<T, 3, 0>(G, r, dinv, omega, i, j + 1, k) + sx;
}

// probe for diag(C^T W C): psi = 1 on the edges of component a whose point is
// congruent to (cx, cy, cz) modulo 3 and not in a wall, 0 elsewhere.  Two
// such edges are three points apart along some axis, so their curls touch
// faces that W does not couple.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_edge_probe(Grid G, int a, int cx, int cy, int cz,
                                                       double* __restrict__ psi) {
  const int k = blockIdx.z;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= G.n[0] * G.n[1]) return;
  const int j = idx / G.n[0], i = idx - j * G.n[0];
  const long nc = G.n_cells;
  const long p = (long)k * G.n[0] * G.n[1] + idx;
  for (int b = 0; b < edge_comps<DIM>(); ++b) {
    const bool on = b == a && i % 3 == cx && j % 3 == cy && (DIM == 2 || k % 3 == cz) &&
                    !edge_in_wall<DIM>(G, b, i, j, k);
    psi[b * nc + p] = on ? 1.0 : 0.0;
  }
}

// diag[e] = t[e] on the probed edges (psi[e] != 0)
__global__ __launch_bounds__(kBlock) void k_edge_collect(long n, const double* __restrict__ psi,
                                                         const double* __restrict__ t,
                                                         double* __restrict__ diag) {
  for (long e = (long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long)gridDim.x * kBlock)
    if (psi[e] != 0.0) diag[e] = t[e];
}

}  // namespace gkb
