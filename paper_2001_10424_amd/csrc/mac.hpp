// MAC (staggered) grid description and matrix-free stencils for gfx950.
//
// Operators (strong-form scaling, cell size h):
//   W  : component-wise -div(mu grad u_c).  Normal-direction couplings use the
//        viscosity of the cell between the two faces, tangential couplings the
//        arithmetic mean of the cells touching the edge between them (edge
//        arrays precomputed on the host).  DIRICHLET side: wall-normal faces
//        are not unknowns (read as 0), tangential wall ghost = -u_f (diagonal
//        gets 2 kappa).  NATURAL side: wall-normal faces are unknowns with half
//        a control volume (tangential terms weighted 1/2), no coupling across.
//   A  : gradient (p_R - p_L)/h on unknown faces; missing or pinned cells = 0.
//   A^T: -div, the exact transpose of A.
//   M  : W + eta A A^T  (augmented Lagrangian with N = I/eta; paper Section 2).
//
// Data layout: velocity full-face SoA u[nz][ny][nx+1], v[nz][ny+1][nx],
// w[nz+1][ny][nx] (x fastest), pressure cells [nz][ny][nx].
#pragma once
#include <hip/hip_runtime.h>

namespace gkb {

constexpr int kDir = 0;
constexpr int kNat = 1;

struct Grid {
  int dim;
  int n[3];       // cells per axis; n[2] = 1 in 2D
  int bc[6];
  int pin;        // flat cell index or -1
  int off[3];     // offset of each component's face array
  int ext[3][3];  // ext[c][a]: extent of component c's array along axis a
  int m_full;
  int n_cells;
  int nze;        // z-extent of the tallest face array: n[2] + (dim == 3)
  double h;
};

inline Grid make_grid(int dim, const int n[3], double h, const int bc[6], int pin) {
  Grid g{};
  g.dim = dim;
  g.n[0] = n[0];
  g.n[1] = n[1];
  g.n[2] = dim == 3 ? n[2] : 1;
  for (int s = 0; s < 6; ++s) g.bc[s] = bc[s];
  if (dim == 2) g.bc[4] = g.bc[5] = kDir;
  g.pin = pin;
  int o = 0;
  for (int c = 0; c < 3; ++c) {
    for (int a = 0; a < 3; ++a) g.ext[c][a] = g.n[a] + ((a == c) ? 1 : 0);
    g.off[c] = o;
    if (c < dim) o += g.ext[c][0] * g.ext[c][1] * g.ext[c][2];
  }
  g.m_full = o;
  g.n_cells = g.n[0] * g.n[1] * g.n[2];
  g.nze = g.n[2] + (dim == 3 ? 1 : 0);
  g.h = h;
  return g;
}

// Coefficients of one grid level in working precision T.
template <typename T>
struct Op {
  Grid g;
  T eta;        // 0 => M = W
  T ih2;        // 1/h^2
  T ih;         // 1/h
  const T* mu;  // cell viscosity (nullptr => 1)
  const T* mue[3];  // edge viscosity, edges parallel to axis b (nullptr => 1)
};

// ------------------------------------------------------------------ helpers

template <int C>
__device__ __forceinline__ int fidx(const Grid& G, int i, int j, int k) {
  return G.off[C] + (k * G.ext[C][1] + j) * G.ext[C][0] + i;
}

__device__ __forceinline__ int cidx(const Grid& G, int i, int j, int k) {
  return (k * G.n[1] + j) * G.n[0] + i;
}

// is the face of component C with normal index ic an unknown?
template <int C>
__device__ __forceinline__ bool unk(const Grid& G, int ic) {
  return !((ic == 0 && G.bc[2 * C] == kDir) || (ic == G.n[C] && G.bc[2 * C + 1] == kDir));
}

template <int C, typename T>
__device__ __forceinline__ T ldm(const Grid& G, const T* __restrict__ x, int i, int j, int k) {
  const int ic = C == 0 ? i : (C == 1 ? j : k);
  return unk<C>(G, ic) ? x[fidx<C>(G, i, j, k)] : T(0);
}

// unscaled cell divergence sum_c (x_lower - x_upper) = h (A^T x)_cell
template <int DIM, typename T>
__device__ __forceinline__ T cdiv(const Grid& G, const T* __restrict__ x, int i, int j, int k) {
  if (cidx(G, i, j, k) == G.pin) return T(0);
  T s = ldm<0>(G, x, i, j, k) - ldm<0>(G, x, i + 1, j, k);
  s += ldm<1>(G, x, i, j, k) - ldm<1>(G, x, i, j + 1, k);
  if (DIM == 3) s += ldm<2>(G, x, i, j, k) - ldm<2>(G, x, i, j, k + 1);
  return s;
}

// viscosity of the edge parallel to axis B at (vertex coords along the other
// two axes, cell coord along B) given as E[0..2]
template <int B, typename T>
__device__ __forceinline__ T edge_mu(const Op<T>& op, int e0, int e1, int e2) {
  const Grid& G = op.g;
  const int x0 = G.n[0] + (B != 0), x1 = G.n[1] + (B != 1);
  return op.mue[B][(e2 * x1 + e1) * x0 + e0];
}

// Row of M (and its diagonal) at the unknown face (C; i, j, k).
template <typename T, int DIM, bool VARMU, int C>
__device__ __forceinline__ void stencil_M(const Op<T>& op, const T* __restrict__ x, int i, int j,
                                          int k, T& Mx, T& dg) {
  const Grid& G = op.g;
  int P[3] = {i, j, k};
  const T xf = x[fidx<C>(G, i, j, k)];
  T acc = T(0), d = T(0);
  const int nC = G.n[C];
  // normal direction: cells P[C]-1 (below) and P[C] (above)
  if (P[C] > 0) {
    int Q[3] = {i, j, k};
    Q[C] -= 1;
    const T kap = VARMU ? op.mu[cidx(G, Q[0], Q[1], Q[2])] : T(1);
    acc += kap * (xf - ldm<C>(G, x, Q[0], Q[1], Q[2]));
    d += kap;
  }
  if (P[C] < nC) {
    int Q[3] = {i, j, k};
    Q[C] += 1;
    const T kap = VARMU ? op.mu[cidx(G, i, j, k)] : T(1);
    acc += kap * (xf - ldm<C>(G, x, Q[0], Q[1], Q[2]));
    d += kap;
  }
  // tangential directions
  const T wgt = (P[C] == 0 || P[C] == nC) ? T(0.5) : T(1);
#pragma unroll
  for (int A = 0; A < DIM; ++A) {
    if (A == C) continue;
    const int B = (DIM == 2) ? 2 : 3 - C - A;
    const int nA = G.n[A];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int e = P[A] + s;  // vertex coordinate of the edge along A
      T kap = T(1);
      if (VARMU) {
        int E[3] = {P[0], P[1], P[2]};
        E[A] = e;  // E[C] = P[C] (vertex), E[B] = P[B] (cell)
        if (B == 0) kap = edge_mu<0>(op, E[0], E[1], E[2]);
        else if (B == 1) kap = edge_mu<1>(op, E[0], E[1], E[2]);
        else kap = edge_mu<2>(op, E[0], E[1], E[2]);
      }
      const int q = s ? P[A] + 1 : P[A] - 1;
      if (q >= 0 && q < nA) {
        int Q[3] = {i, j, k};
        Q[A] = q;
        acc += wgt * kap * (xf - x[fidx<C>(G, Q[0], Q[1], Q[2])]);
        d += wgt * kap;
      } else if (G.bc[2 * A + s] == kDir) {
        acc += T(2) * wgt * kap * xf;
        d += T(2) * wgt * kap;
      }
    }
  }
  // grad-div: eta A A^T x = eta (div_R - div_L) / h^2 with div = h A^T x
  if (op.eta != T(0)) {
    T tR = T(0), tL = T(0);
    int cnt = 0;
    if (P[C] < nC) {
      tR = cdiv<DIM>(G, x, i, j, k);
      cnt += cidx(G, i, j, k) != G.pin;
    }
    if (P[C] > 0) {
      int Q[3] = {i, j, k};
      Q[C] -= 1;
      tL = cdiv<DIM>(G, x, Q[0], Q[1], Q[2]);
      cnt += cidx(G, Q[0], Q[1], Q[2]) != G.pin;
    }
    acc += op.eta * (tR - tL);
    d += op.eta * T(cnt);
  }
  Mx = acc * op.ih2;
  dg = d * op.ih2;
}

// Diagonal of M at the unknown face (C; i, j, k) without touching x.
template <typename T, int DIM, bool VARMU, int C>
__device__ __forceinline__ T diag_M(const Op<T>& op, int i, int j, int k) {
  const Grid& G = op.g;
  int P[3] = {i, j, k};
  T d = T(0);
  const int nC = G.n[C];
  if (P[C] > 0) {
    int Q[3] = {i, j, k};
    Q[C] -= 1;
    d += VARMU ? op.mu[cidx(G, Q[0], Q[1], Q[2])] : T(1);
  }
  if (P[C] < nC) d += VARMU ? op.mu[cidx(G, i, j, k)] : T(1);
  const T wgt = (P[C] == 0 || P[C] == nC) ? T(0.5) : T(1);
#pragma unroll
  for (int A = 0; A < DIM; ++A) {
    if (A == C) continue;
    const int B = (DIM == 2) ? 2 : 3 - C - A;
    const int nA = G.n[A];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int e = P[A] + s;
      T kap = T(1);
      if (VARMU) {
        int E[3] = {P[0], P[1], P[2]};
        E[A] = e;
        if (B == 0) kap = edge_mu<0>(op, E[0], E[1], E[2]);
        else if (B == 1) kap = edge_mu<1>(op, E[0], E[1], E[2]);
        else kap = edge_mu<2>(op, E[0], E[1], E[2]);
      }
      const int q = s ? P[A] + 1 : P[A] - 1;
      if (q >= 0 && q < nA) d += wgt * kap;
      else if (G.bc[2 * A + s] == kDir) d += T(2) * wgt * kap;
    }
  }
  if (op.eta != T(0)) {
    int cnt = 0;
    if (P[C] < nC) cnt += cidx(G, i, j, k) != G.pin;
    if (P[C] > 0) {
      int Q[3] = {i, j, k};
      Q[C] -= 1;
      cnt += cidx(G, Q[0], Q[1], Q[2]) != G.pin;
    }
    d += op.eta * T(cnt);
  }
  return d * op.ih2;
}

// (A p)_f at the unknown face (C; i, j, k)
template <int C, typename T>
__device__ __forceinline__ T grad_f(const Grid& G, const T* __restrict__ p, int i, int j, int k) {
  int P[3] = {i, j, k};
  T pr = T(0), pl = T(0);
  if (P[C] < G.n[C] && cidx(G, i, j, k) != G.pin) pr = p[cidx(G, i, j, k)];
  if (P[C] > 0) {
    int Q[3] = {i, j, k};
    Q[C] -= 1;
    const int cq = cidx(G, Q[0], Q[1], Q[2]);
    if (cq != G.pin) pl = p[cq];
  }
  return pr - pl;  // caller scales by 1/h
}

}  // namespace gkb
