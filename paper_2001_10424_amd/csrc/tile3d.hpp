// LDS-tiled 3D MAC stencil for M = W + eta A A^T (and the Jacobi / residual
// variants built on it) on grids whose +x, +y, +z sides are DIRICHLET.
//
// A block of 256 threads (4 wave64) owns a tile of 64 x 4 cells in x-y and
// marches through `tz` consecutive z-planes.  Each thread owns one x
// position and kRPT y rows and produces the three "lower" faces u(i,j,k),
// v(i,j,k), w(i,j,k) of its cells; the upper boundary faces (i = nx, ...)
// are Dirichlet faces and are written as 0 by the last row / column / plane.
//
// Per z-plane the block stages the face values of the plane k+1 of u, v, w
// for the tile plus a one-cell halo in a two-slot LDS ring (plane k is
// already there), computes the cell divergence of plane k for the tile plus
// its lower halo row/column once into LDS (it feeds the grad-div term of up
// to six faces), and keeps the plane k-1 values of its own faces and the
// divergence of its cell below in registers.  Global traffic per plane is one
// pass over the tile (+ halo, mostly L2 hits) of x, plus b and y for the
// faces the block owns.
//
// Two modes transform the values while they are staged, so that a V-cycle
// step needs no separate pass over memory: kJacobiZ stages x1 = omega b / D
// (the first sweep from a zero guess; the kernel then applies the second),
// and kJacobiP stages x + P e, the prolongation of the coarse-grid
// correction e.
#pragma once
#include "kernels.hpp"

namespace gkb {

constexpr int kTX = 64;          // tile width (cells) = threads in x
constexpr int kTYT = 256 / kTX;  // threads in y
// rows per thread: one row (64 x 4 tiles, 8 planes per block at 128^3)
// measured 4% faster in FP32 and 5% in FP64 than two rows (64 x 8 tiles,
// 4 planes per block): half the per-thread state, the per-block set-up
// spread over twice the planes
constexpr int kRPT = 1;
constexpr int kTY = kTYT * kRPT; // tile height (cells)
constexpr int kLX = kTX + 2;
constexpr int kLY = kTY + 2;

template <typename T>
struct TileLds {
  T u[2][kLY][kLX];
  T v[2][kLY][kLX];
  T w[2][kLY][kLX];
  T cd[kTY + 1][kTX + 1];
};

// one axis of the viscous stencil; lo_in / hi_in: neighbour inside the array,
// lo_wall / hi_wall: neighbour across a DIRICHLET wall (mirror ghost).
// Branch-free: the neighbour values outside the array are zeros in LDS, so
// their coefficients are selected instead of branched on.
template <typename T>
__device__ __forceinline__ void visc_axis(T xf, T vlo, T vhi, bool lo_in, bool hi_in, bool lo_wall,
                                          bool hi_wall, T klo, T khi, T wgt, T& acc, T& d) {
  const T wlo = wgt * klo, whi = wgt * khi;
  const T clo = lo_in ? wlo : T(0), chi = hi_in ? whi : T(0);
  const T alo = lo_in ? wlo : (lo_wall ? T(2) * wlo : T(0));
  const T ahi = hi_in ? whi : (hi_wall ? T(2) * whi : T(0));
  acc += (alo + ahi) * xf - clo * vlo - chi * vhi;
  d += alo + ahi;
}

// 1 / d for the Jacobi step: the hardware reciprocal in FP32 (about 1 ulp,
// plenty for a smoother), exact division in FP64
template <typename T>
__device__ __forceinline__ T recip(T d) {
  return T(1) / d;
}
template <>
__device__ __forceinline__ float recip<float>(float d) {
  return __builtin_amdgcn_rcpf(d);
}

// Raw buffer access: a scalar base (buffer resource) plus a per-lane 32-bit
// byte offset and a uniform scalar byte offset, so an access costs no 64-bit
// address arithmetic.  The tiled kernel is used only for face arrays below
// 2 GiB, which keeps every offset in 31 bits.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                 unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                   unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}

template <int MODE>
constexpr bool reads_b() {
  return MODE == kJacobi || MODE == kJacobiDot || MODE == kResid || MODE == kResidDot ||
         MODE == kJacobiZ || MODE == kJacobiP;
}

// bf: b at the face (prefetched by the caller when the mode reads b); unk:
// the face is an unknown (else 0 is written, computed values discarded);
// the result goes to byte offset voff + soff of y
template <typename T, int MODE>
__device__ __forceinline__ double tile_finish(unsigned voff, unsigned soff, bool unk, T mx, T d,
                                              T xf, T bf, __amdgpu_buffer_rsrc_t ry, T omega,
                                              __amdgpu_buffer_rsrc_t ry2) {
  double part = 0.0;
  T out;
  if (MODE == kApply || MODE == kApplyDot || MODE == kApplyDotP) {
    out = unk ? mx : T(0);
    if (MODE == kApplyDot || MODE == kApplyDotP) part = double(xf) * double(out);
  } else if (MODE == kJacobi || MODE == kJacobiDot || MODE == kJacobiZ || MODE == kJacobiP) {
    out = unk ? xf + omega * (bf - mx) * recip(d) : T(0);
    if (MODE == kJacobiDot) part = double(bf) * double(out);
  } else if (MODE == kResid || MODE == kResidDot) {
    out = unk ? bf - mx : T(0);
    if (MODE == kResidDot) part = double(out) * double(out);
  } else {  // kDinvM
    out = unk ? mx * recip(d) : T(0);
    part = double(out) * double(out);
  }
  buf_store(out, ry, voff, soff);
  if (MODE == kApplyDotP) buf_store(unk ? xf : T(0), ry2, voff, soff);  // p'
  return part;
}

// Constant-viscosity variant of tile_finish: mx = (M x) at the face and sc
// the hoisted diagonal scale (omega / D for the Jacobi modes, 1 / D for
// kDinvM, unused otherwise).
template <typename T, int MODE>
__device__ __forceinline__ double tile_out(unsigned voff, unsigned soff, bool unk, T mx, T sc,
                                           T xf, T bf, __amdgpu_buffer_rsrc_t ry,
                                           __amdgpu_buffer_rsrc_t ry2) {
  double part = 0.0;
  T out;
  if (MODE == kApply || MODE == kApplyDot || MODE == kApplyDotP) {
    out = unk ? mx : T(0);
    if (MODE == kApplyDot || MODE == kApplyDotP) part = double(xf) * double(out);
  } else if (MODE == kJacobi || MODE == kJacobiDot || MODE == kJacobiZ || MODE == kJacobiP) {
    out = unk ? xf + (bf - mx) * sc : T(0);
    if (MODE == kJacobiDot) part = double(bf) * double(out);
  } else if (MODE == kResid || MODE == kResidDot) {
    out = unk ? bf - mx : T(0);
    if (MODE == kResidDot) part = double(out) * double(out);
  } else {  // kDinvM
    out = unk ? mx * sc : T(0);
    part = double(out) * double(out);
  }
  buf_store(out, ry, voff, soff);
  if (MODE == kApplyDotP) buf_store(unk ? xf : T(0), ry2, voff, soff);  // p'
  return part;
}

// diagonal count of one axis of the viscous stencil: an in-array neighbour
// counts 1, a DIRICHLET wall across the face (mirror ghost) 2, else 0
__device__ __forceinline__ int axis_count(bool lo_in, bool hi_in, bool lo_wall, bool hi_wall) {
  return (lo_in ? 1 : (lo_wall ? 2 : 0)) + (hi_in ? 1 : (hi_wall ? 2 : 0));
}

// Diagonal of M times h^2 (the caller applies 1/h^2) at
// the face (component c; i, j, k) for constant viscosity, branch-free: the
// viscous counts of the normal and the two tangential axes (tangential ones
// halved on a boundary-normal face) plus eta times the number of valid
// adjacent cells; (pi, pj, pk) is the pinned cell.
template <typename T>
__device__ __forceinline__ T diag_const(const Grid& G, T eta, int c, int i, int j, int k, int pi,
                                        int pj, int pk) {
  const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
  const int cx = axis_count(i > 0, i < n0 - 1, G.bc[0] == kDir, G.bc[1] == kDir);
  const int cy = axis_count(j > 0, j < n1 - 1, G.bc[2] == kDir, G.bc[3] == kDir);
  const int cz = axis_count(k > 0, k < n2 - 1, G.bc[4] == kDir, G.bc[5] == kDir);
  const int P = c == 0 ? i : (c == 1 ? j : k), N = c == 0 ? n0 : (c == 1 ? n1 : n2);
  const int normal = int(P > 0) + int(P < N);
  const int tang = c == 0 ? cy + cz : (c == 1 ? cx + cz : cx + cy);
  const T wgt = (P == 0 || P == N) ? T(0.5) : T(1);
  // adjacent cells along the normal: (i, j, k) and the one below it
  const bool at_pin = i == pi && j == pj && k == pk;
  const bool below_pin = (c == 0 ? (i - 1 == pi && j == pj && k == pk)
                                 : (c == 1 ? (i == pi && j - 1 == pj && k == pk)
                                           : (i == pi && j == pj && k - 1 == pk)));
  const int cnt = int(P < N && !at_pin) + int(P > 0 && !below_pin);
  return T(normal) + wgt * T(tang) + eta * T(cnt);
}

// FINE only separates the finest-grid launches from the coarse-level ones in
// kernel traces; the code is the same.
//
// Latency hiding: every global load is unconditional from an address that is
// always valid (indices outside the grid or on non-unknown faces are clamped
// to the first entry of the array) and the mask is applied when the value is
// stored to LDS, so no load sits under a branch.  Loads run two planes ahead:
// while plane k is computed, the x values of plane k+2 and b of plane k+1 are
// already in flight and plane k+3 (x) and k+2 (b) are issued.  Two register
// sets of each take turns (the plane loop is unrolled by two), so consuming
// one never waits for the loads into the other; the prologue issues its four
// planes at once.
// FP32: at least 4 waves per SIMD (4 blocks per CU, all of the 128^3 grid
// in one round; the one-row kernels need about 85 VGPRs, so the cap does not
// bind, and 6 waves per SIMD measured no faster); FP64 runs uncapped
template <typename T>
constexpr int kTileMinWaves = sizeof(T) == 4 ? 4 : 1;

template <typename T, bool VARMU, int MODE, bool FINE>
__global__ __launch_bounds__(256, kTileMinWaves<T>) void k_tile3d(Op<T> op, const T* __restrict__ x,
                                                const T* __restrict__ b, T* __restrict__ y,
                                                T omega, int tz, double* __restrict__ partial,
                                                const PcgState* __restrict__ st,
                                                const T* __restrict__ ec, Grid Gc,
                                                T* __restrict__ y2) {
  if (st && st->done) return;
  __shared__ TileLds<T> S;
  const Grid& G = op.g;
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  // XCD-aware block order: consecutive logical tiles on the same XCD
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  int lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  if ((nb & 7) == 0) lin = (lin & 7) * (nb >> 3) + (lin >> 3);
  const int bx = lin % gridDim.x;
  const int rest = lin / gridDim.x;
  const int by = rest % gridDim.y, bz = rest / gridDim.y;
  const int i0 = bx * kTX, j0 = by * kTY, k0 = bz * tz;
  const int k1 = min(k0 + tz, nz);
  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const bool unk_u0 = G.bc[0] == kNat, unk_v0 = G.bc[2] == kNat, unk_w0 = G.bc[4] == kNat;
  // plane strides of the three face arrays
  const int pu = G.ext[0][0] * G.ext[0][1], pv = G.ext[1][0] * G.ext[1][1],
            pw = G.ext[2][0] * G.ext[2][1];
  constexpr unsigned E = sizeof(T);
  const unsigned bytes = unsigned(G.m_full) * E;
  const __amdgpu_buffer_rsrc_t rx = buf_rsrc(x, bytes), ry = buf_rsrc(y, bytes);
  const __amdgpu_buffer_rsrc_t rb = reads_b<MODE>() ? buf_rsrc(b, bytes) : rx;
  // w-array offset relative to the v array (same in-plane index: both are
  // nx wide), added to the uniform part of a w access
  const unsigned dw = unsigned(G.off[2] - G.off[1]) * E;

  // staged halo elements of this thread: in-plane byte offset (clamped) and
  // validity bits (u, v, w per element), fixed for the whole block
  constexpr int kPer = (kLX * kLY + 255) / 256;
  unsigned hu[kPer], hv[kPer];
  unsigned hmask = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = threadIdx.x + q * 256;
    const int jj = e / kLX, ii = e - jj * kLX;
    const int i = i0 - 1 + ii, j = j0 - 1 + jj;
    const bool in = e < kLX * kLY && j >= 0 && j < ny && i >= 0 && i < nx;
    const bool ou = in && (i > 0 || unk_u0), ov = in && (j > 0 || unk_v0);
    hu[q] = unsigned(G.off[0] + (ou ? j * G.ext[0][0] + i : 0)) * E;
    // v and w share the in-plane index (both arrays are nx wide): the w
    // offset is the v offset + dw; non-unknown v faces are masked at the
    // LDS store, so the v offset is clamped only outside the grid
    hv[q] = unsigned(G.off[1] + (in ? j * G.ext[1][0] + i : 0)) * E;
    hmask |= (ou ? 1u : 0u) << (3 * q);
    hmask |= (ov ? 2u : 0u) << (3 * q);
    hmask |= (in ? 4u : 0u) << (3 * q);
  }
  // kJacobiP: the staged values are x + P e, the prolongation of the coarse
  // correction e on the grid Gc (a fine face on a coarse face takes its
  // value, a face between two coarse faces their mean; constant across the
  // two fine cells in the tangential directions; non-unknown coarse faces
  // count as 0).  Per staged element: in-plane index of the coarse u and v
  // faces at (i/2, j/2) (w shares v's: both arrays are nx/2 wide) and six
  // bits: odd i, odd j, coarse u faces I and I+1 unknown, coarse v faces J
  // and J+1 unknown.  The coarse values (faces I / I+1, J / J+1, coarse
  // planes K / K+1) are prefetched with the plane; an odd plane k >= k0
  // lies on the coarse plane K of the even plane before it, staged just
  // before it by the same thread, and takes that plane's five values from
  // registers (only the plane K+1 of its w faces is loaded), which halves
  // the coarse loads.
  constexpr bool kP = MODE == kJacobiP;
  // kApplyDotP: the staged values are p' = z + beta p (x = z, b = p); p is
  // loaded with z into the second register set, p' is written to y2 at the
  // block's own faces
  constexpr bool kAP = MODE == kApplyDotP;
  constexpr int kPC = kP ? 6 : (kAP ? 3 : 1);
  const T pbeta = (kAP && st) ? T(st->beta) : T(0);
  const __amdgpu_buffer_rsrc_t rpo = kAP ? buf_rsrc(b, bytes) : rx;
  const __amdgpu_buffer_rsrc_t ry2 = kAP ? buf_rsrc(y2, bytes) : ry;
  unsigned pcu[kPer], pcv[kPer], pbits = 0;
  const __amdgpu_buffer_rsrc_t rc = kP ? buf_rsrc(ec, unsigned(Gc.m_full) * E) : rx;
  const unsigned dwc = kP ? unsigned(Gc.off[2] - Gc.off[1]) * E : 0u;
  if (kP) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = threadIdx.x + q * 256;
      const int jj = e / kLX, ii = e - jj * kLX;
      const int i = i0 - 1 + ii, j = j0 - 1 + jj;
      const bool in = (hmask >> (3 * q + 2)) & 1u;
      const int I = in ? i >> 1 : 0, J = in ? j >> 1 : 0;
      pcu[q] = unsigned(Gc.off[0] + J * Gc.ext[0][0] + I) * E;
      pcv[q] = unsigned(Gc.off[1] + J * Gc.ext[1][0] + I) * E;
      const bool uI = !((I == 0 && Gc.bc[0] == kDir) || (I == Gc.n[0] && Gc.bc[1] == kDir));
      const bool uI1 = !(I + 1 == Gc.n[0] && Gc.bc[1] == kDir);
      const bool vJ = !((J == 0 && Gc.bc[2] == kDir) || (J == Gc.n[1] && Gc.bc[3] == kDir));
      const bool vJ1 = !(J + 1 == Gc.n[1] && Gc.bc[3] == kDir);
      const unsigned bits = (i & 1 ? 1u : 0u) | (j & 1 ? 2u : 0u) | (uI ? 4u : 0u) |
                            (uI1 ? 8u : 0u) | (vJ ? 16u : 0u) | (vJ1 ? 32u : 0u);
      pbits |= bits << (6 * q);
    }
  }
  struct FRegs {
    T v[3][kPer];
    T c[kPC][kPer];  // kJacobiP: coarse u(I), u(I+1), v(J), v(J+1), w(K), w(K+1)
  };
  // kJacobiP: an odd plane after the block's first takes the coarse plane-K
  // values of the even plane staged before it (cprev)
  auto reuse_coarse = [&](int k) { return (k & 1) && k >= k0 && k < nz; };
  T cprev[5][kPer];
  auto fetch_plane = [&](int k, FRegs& F) {
    const int kk = min(max(k, 0), nz - 1);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      F.v[0][q] = buf_load<T>(rx, hu[q], unsigned(kk * pu) * E);
      F.v[1][q] = buf_load<T>(rx, hv[q], unsigned(kk * pv) * E);
      F.v[2][q] = buf_load<T>(rx, hv[q], unsigned(kk * pw) * E + dw);
    }
    if (kAP) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        F.c[0][q] = buf_load<T>(rpo, hu[q], unsigned(kk * pu) * E);
        F.c[1][q] = buf_load<T>(rpo, hv[q], unsigned(kk * pv) * E);
        F.c[2][q] = buf_load<T>(rpo, hv[q], unsigned(kk * pw) * E + dw);
      }
    }
    if (kP) {
      const int K = kk >> 1, K1 = min(K + 1, Gc.ext[2][2] - 1);
      const unsigned su = unsigned(K * Gc.ext[0][0] * Gc.ext[0][1]) * E;
      const unsigned sv = unsigned(K * Gc.ext[1][0] * Gc.ext[1][1]) * E;
      const unsigned sw = unsigned(K * Gc.ext[2][0] * Gc.ext[2][1]) * E + dwc;
      const unsigned sw1 = unsigned(K1 * Gc.ext[2][0] * Gc.ext[2][1]) * E + dwc;
      const unsigned rowv = unsigned(Gc.ext[1][0]) * E;
      if (!reuse_coarse(k)) {  // uniform
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
          F.c[0][q] = buf_load<T>(rc, pcu[q], su);
          F.c[1][q] = buf_load<T>(rc, pcu[q] + E, su);
          F.c[2][q] = buf_load<T>(rc, pcv[q], sv);
          F.c[3][q] = buf_load<T>(rc, pcv[q] + rowv, sv);
          F.c[4][q] = buf_load<T>(rc, pcv[q], sw);
        }
      }
      // the coarse plane above is needed by the w faces of odd planes only
      if (kk & 1) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) F.c[5][q] = buf_load<T>(rc, pcv[q], sw1);
      }
    }
  };
  // pinned cell (pk = -2: none)
  const int nxy = nx * ny;
  const int pk = G.pin >= 0 ? G.pin / nxy : -2;
  const int pj = G.pin >= 0 ? (G.pin - pk * nxy) / nx : -3;
  const int pi = G.pin >= 0 ? G.pin - pk * nxy - pj * nx : -3;

  // kJacobiZ (x = b): the staged values are the first sweep from a zero
  // guess, x1 = omega b / D.  zs holds omega / D of the staged elements for
  // every plane whose diagonal is the bulk one (not the first or last plane,
  // not next to the pinned cell), taken on plane zb (-1: no such plane, the
  // scales are computed per plane); other planes compute them (uniform
  // branch, at most four planes of a grid)
  constexpr bool kZ = MODE == kJacobiZ;
  static_assert(!(kZ && VARMU), "the two-sweep mode is for constant viscosity");
  auto zbulk = [&](int k) { return k > 0 && k < nz - 1 && k != pk && k - 1 != pk; };
  auto zscale = [&](int q, int c, int k) -> T {
    const int e = threadIdx.x + q * 256;
    const int jj = e / kLX, ii = e - jj * kLX;
    const int i = i0 - 1 + ii, j = j0 - 1 + jj;
    if (!((hmask >> (3 * q + c)) & 1u)) return T(0);  // not staged: any value
    return omega * recip(diag_const<T>(G, op.eta, c, i, j, k, pi, pj, pk) * op.ih2);
  };
  int zb = -1;
  T zs[3][kPer];
  if (kZ) {
    for (int kk = 1; kk < min(nz - 1, 4) && zb < 0; ++kk)
      if (zbulk(kk)) zb = kk;
#pragma unroll
    for (int q = 0; q < kPer; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) zs[c][q] = zb >= 0 ? zscale(q, c, zb) : T(0);
  }
  auto store_plane = [&](int s, int k, const FRegs& F) {
    const bool kin = k >= 0 && k < nz;
    const bool kw = kin && (k > 0 || unk_w0);
    T val[3][kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) val[c][q] = kAP ? F.v[c][q] + pbeta * F.c[c][q] : F.v[c][q];
    if (kP && kin) {
      // coarse plane K = k / 2; a w face on an odd plane lies between K and K+1
      const int K = k >> 1;
      const bool wK = !((K == 0 && Gc.bc[4] == kDir) || (K == Gc.n[2] && Gc.bc[5] == kDir));
      const bool wK1 = !(K + 1 == Gc.n[2] && Gc.bc[5] == kDir);
      const bool oddk = k & 1;
      const bool reuse = reuse_coarse(k);  // uniform
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        T cv[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          cv[c] = reuse ? cprev[c][q] : F.c[c][q];
          cprev[c][q] = cv[c];
        }
        const unsigned bq = pbits >> (6 * q);
        const T u0 = (bq & 4u) ? cv[0] : T(0), u1 = (bq & 8u) ? cv[1] : T(0);
        const T v0 = (bq & 16u) ? cv[2] : T(0), v1 = (bq & 32u) ? cv[3] : T(0);
        const T w0 = wK ? cv[4] : T(0), w1 = wK1 ? F.c[5][q] : T(0);
        val[0][q] += (bq & 1u) ? T(0.5) * (u0 + u1) : u0;
        val[1][q] += (bq & 2u) ? T(0.5) * (v0 + v1) : v0;
        val[2][q] += oddk ? T(0.5) * (w0 + w1) : w0;
      }
    }
    T z[3][kPer];
    if (kZ) {
      if (zb >= 0 && zbulk(k)) {
#pragma unroll
        for (int q = 0; q < kPer; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) z[c][q] = zs[c][q];
      } else {
#pragma unroll
        for (int q = 0; q < kPer; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) z[c][q] = kin ? zscale(q, c, k) : T(0);
      }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = threadIdx.x + q * 256;
      if (e < kLX * kLY) {
        const int jj = e / kLX, ii = e - jj * kLX;
        const unsigned m = hmask >> (3 * q);
        S.u[s][jj][ii] = (kin && (m & 1u)) ? (kZ ? val[0][q] * z[0][q] : val[0][q]) : T(0);
        S.v[s][jj][ii] = (kin && (m & 2u)) ? (kZ ? val[1][q] * z[1][q] : val[1][q]) : T(0);
        S.w[s][jj][ii] = (kw && (m & 4u)) ? (kZ ? val[2][q] * z[2][q] : val[2][q]) : T(0);
      }
    }
  };
  auto cell_ok = [&](int i, int j, int k) {
    return i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz && cidx(G, i, j, k) != G.pin;
  };

  // this thread's faces: in-plane byte offset of u and v (w: v + dw), clamped
  // when outside
  unsigned fo[kRPT][2];
#pragma unroll
  for (int r = 0; r < kRPT; ++r) {
    const int i = i0 + tx, j = j0 + ty + r * kTYT;
    const bool in = i < nx && j < ny;
    fo[r][0] = unsigned(G.off[0] + (in ? j * G.ext[0][0] + i : 0)) * E;
    fo[r][1] = unsigned(G.off[1] + (in ? j * G.ext[1][0] + i : 0)) * E;
  }
  typedef T BRegs[kRPT][3];
  auto fetch_b = [&](int k, BRegs& bb) {
    if (!reads_b<MODE>()) return;
    const int kk = min(k, nz - 1);
#pragma unroll
    for (int r = 0; r < kRPT; ++r) {
      bb[r][0] = buf_load<T>(rb, fo[r][0], unsigned(kk * pu) * E);
      bb[r][1] = buf_load<T>(rb, fo[r][1], unsigned(kk * pv) * E);
      bb[r][2] = buf_load<T>(rb, fo[r][1], unsigned(kk * pw) * E + dw);
    }
  };


  // Constant viscosity: the neighbours outside the array and the
  // non-unknown faces are zeros in LDS and in the z registers, so the
  // off-diagonal part of every face is the plain weighted sum of its six
  // neighbours; the diagonal (viscous count + eta x number of valid adjacent
  // cells) changes with z only on the first and last plane and next to the
  // pinned cell.  dv: viscous diagonal count, sc: omega / D (Jacobi modes)
  // or 1 / D, for plane k, or (bulk) for any plane away from those.
  T dv[kRPT][3], sc[kRPT][3];
  auto coef = [&](int k, bool bulk) {
    const int czt = bulk ? 2 : axis_count(k > 0, k < nz - 1, G.bc[4] == kDir, G.bc[5] == kDir);
    const int cnw = bulk ? 2 : int(k > 0) + 1;
    const T ww = (!bulk && k == 0) ? T(0.5) : T(1);
    const bool pz = !bulk && k == pk, pz1 = !bulk && k - 1 == pk, kpos = bulk || k > 0;
#pragma unroll
    for (int r = 0; r < kRPT; ++r) {
      const int i = i0 + tx, j = j0 + ty + r * kTYT;
      const bool pc = i == pi && j == pj, pl = i - 1 == pi && j == pj, ps = i == pi && j - 1 == pj;
      const int cx = axis_count(i > 0, i < nx - 1, G.bc[0] == kDir, G.bc[1] == kDir);
      const int cy = axis_count(j > 0, j < ny - 1, G.bc[2] == kDir, G.bc[3] == kDir);
      const T wu = i == 0 ? T(0.5) : T(1), wv = j == 0 ? T(0.5) : T(1);
      dv[r][0] = T(int(i > 0) + 1) + wu * T(cy + czt);
      dv[r][1] = T(int(j > 0) + 1) + wv * T(cx + czt);
      dv[r][2] = T(cnw) + ww * T(cx + cy);
      const int own = int(!(pz && pc));
      const int ncell[3] = {own + int(i > 0 && !(pz && pl)), own + int(j > 0 && !(pz && ps)),
                            own + int(kpos && !(pz1 && pc))};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T dt = (dv[r][c] + op.eta * T(ncell[c])) * op.ih2;
        sc[r][c] = (MODE == kJacobi || MODE == kJacobiDot || MODE == kJacobiZ || MODE == kJacobiP)
                       ? omega * recip(dt)
                       : recip(dt);
      }
    }
  };
  // Constant viscosity: each thread takes the divergence of its own cells
  // from the face values it reads for its faces anyway; the 73 halo cells of
  // the tile go to the threads t < 73: t <= 64 the row j0 - 1 (cell
  // i0 - 1 + t), t = 65..72 the column i0 - 1 (row j0 - 1 + t - 64).
  // (hcj, hci): that cell in the divergence array; hbits bit 0: it exists,
  // bit 1: it lies in the pinned cell's column, bit 2 + r: the thread's own
  // cell of row r lies in that column.
  int hci = 0, hcj = 0;
  unsigned hbits = 0;
  if (!VARMU) {
    const int t = threadIdx.x;
    hci = t < kTX + 1 ? t : 0;
    hcj = t < kTX + 1 ? 0 : t - kTX;
    const int i = i0 - 1 + hci, j = j0 - 1 + hcj;
    const bool ok = t < kTX + 1 + kTY && i >= 0 && i < nx && j >= 0 && j < ny;
    hbits = (ok ? 1u : 0u) | (ok && i == pi && j == pj ? 2u : 0u);
#pragma unroll
    for (int r = 0; r < kRPT; ++r)
      hbits |= (i0 + tx == pi && j0 + ty + r * kTYT == pj ? 4u : 0u) << r;
    coef(0, true);
  }

  T up[kRPT], vp[kRPT], wp[kRPT], cdp[kRPT];
  BRegs bA, bB;
#pragma unroll
  for (int r = 0; r < kRPT; ++r)
    bA[r][0] = bA[r][1] = bA[r][2] = bB[r][0] = bB[r][1] = bB[r][2] = T(0);
  FRegs FA, FB;
  fetch_plane(k0 - 1, FA);
  fetch_plane(k0, FB);
  store_plane(1, k0 - 1, FA);
  store_plane(0, k0, FB);
  // planes k0+1 (FA) and k0+2 (FB), b of planes k0 (bA) and k0+1 (bB)
  // (prefetches past the block's last plane re-read its last plane, a cache
  // hit: issuing them unconditionally keeps the number of loads in flight
  // fixed, so each wait can leave the younger prefetches outstanding)
  fetch_plane(k0 + 1, FA);
  fetch_plane(min(k0 + 2, k1), FB);
  fetch_b(k0, bA);
  fetch_b(min(k0 + 1, k1 - 1), bB);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRPT; ++r) {
    const int jj = ty + r * kTYT + 1, ii = tx + 1;
    const int i = i0 + tx, j = j0 + ty + r * kTYT;
    up[r] = S.u[1][jj][ii];
    vp[r] = S.v[1][jj][ii];
    wp[r] = S.w[1][jj][ii];
    cdp[r] = cell_ok(i, j, k0 - 1)
                 ? (S.u[1][jj][ii] - S.u[1][jj][ii + 1] + S.v[1][jj][ii] - S.v[1][jj + 1][ii] +
                    S.w[1][jj][ii] - S.w[0][jj][ii])
                 : T(0);
  }
  __syncthreads();

  const T eta = op.eta, ih2 = op.ih2;
  double part = 0.0;
  // one z-plane (variable viscosity): x of plane k+1 is in F and b of plane
  // k in bc; F is refilled with plane k+3 and bc with b of plane k+2
  auto step = [&](int k, FRegs& F, BRegs& bc) {
    const int s = (k - k0) & 1, s1 = s ^ 1;
    store_plane(s1, k + 1, F);
    __syncthreads();
    fetch_plane(min(k + 3, k1), F);
    // divergence sums of plane k for cells (i0-1 .. i0+63) x (j0-1 .. j0+7)
    for (int e = threadIdx.x; e < (kTX + 1) * (kTY + 1); e += 256) {
      const int cj = e / (kTX + 1), ci = e - cj * (kTX + 1);
      const int i = i0 - 1 + ci, j = j0 - 1 + cj;
      T v = T(0);
      if (cell_ok(i, j, k))
        v = S.u[s][cj][ci] - S.u[s][cj][ci + 1] + S.v[s][cj][ci] - S.v[s][cj + 1][ci] +
            S.w[s][cj][ci] - S.w[s1][cj][ci];
      S.cd[cj][ci] = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRPT; ++r) {
      const int jj = ty + r * kTYT + 1, ii = tx + 1;
      const int i = i0 + tx, j = j0 + ty + r * kTYT;
      if (i < nx && j < ny) {
        const T cR = S.cd[jj][ii];
        const bool okR = cell_ok(i, j, k);
        // ---- u-face (i, j, k): normal x
        {
          {
            const T xf = S.u[s][jj][ii];
            T acc = T(0), d = T(0);
            T kn0 = T(1), kn1 = T(1), ky0 = T(1), ky1 = T(1), kz0 = T(1), kz1 = T(1);
            if (VARMU) {
              kn0 = op.mu[cidx(G, max(i - 1, 0), j, k)];
              kn1 = op.mu[cidx(G, i, j, k)];
              ky0 = edge_mu<2>(op, i, j, k);
              ky1 = edge_mu<2>(op, i, j + 1, k);
              kz0 = edge_mu<1>(op, i, j, k);
              kz1 = edge_mu<1>(op, i, j, k + 1);
            }
            visc_axis<T>(xf, S.u[s][jj][ii - 1], S.u[s][jj][ii + 1], i > 0, true, false, false,
                         kn0, kn1, T(1), acc, d);
            const T wgt = (i == 0) ? T(0.5) : T(1);
            visc_axis<T>(xf, S.u[s][jj - 1][ii], S.u[s][jj + 1][ii], j > 0, j < ny - 1,
                         G.bc[2] == kDir, G.bc[3] == kDir, ky0, ky1, wgt, acc, d);
            visc_axis<T>(xf, up[r], S.u[s1][jj][ii], k > 0, k < nz - 1, G.bc[4] == kDir,
                         G.bc[5] == kDir, kz0, kz1, wgt, acc, d);
            if (eta != T(0)) {
              const T cL = S.cd[jj][ii - 1];
              const int cnt = int(okR) + int(cell_ok(i - 1, j, k));
              acc += eta * (cR - cL);
              d += eta * T(cnt);
            }
            part += tile_finish<T, MODE>(fo[r][0], unsigned(k * pu) * E, i > 0 || unk_u0,
                                         acc * ih2, d * ih2, xf, bc[r][0], ry, omega, ry2);
          }
        }
        // ---- v-face (i, j, k): normal y
        {
          {
            const T xf = S.v[s][jj][ii];
            T acc = T(0), d = T(0);
            T kn0 = T(1), kn1 = T(1), kx0 = T(1), kx1 = T(1), kz0 = T(1), kz1 = T(1);
            if (VARMU) {
              kn0 = op.mu[cidx(G, i, max(j - 1, 0), k)];
              kn1 = op.mu[cidx(G, i, j, k)];
              kx0 = edge_mu<2>(op, i, j, k);
              kx1 = edge_mu<2>(op, i + 1, j, k);
              kz0 = edge_mu<0>(op, i, j, k);
              kz1 = edge_mu<0>(op, i, j, k + 1);
            }
            visc_axis<T>(xf, S.v[s][jj - 1][ii], S.v[s][jj + 1][ii], j > 0, true, false, false,
                         kn0, kn1, T(1), acc, d);
            const T wgt = (j == 0) ? T(0.5) : T(1);
            visc_axis<T>(xf, S.v[s][jj][ii - 1], S.v[s][jj][ii + 1], i > 0, i < nx - 1,
                         G.bc[0] == kDir, G.bc[1] == kDir, kx0, kx1, wgt, acc, d);
            visc_axis<T>(xf, vp[r], S.v[s1][jj][ii], k > 0, k < nz - 1, G.bc[4] == kDir,
                         G.bc[5] == kDir, kz0, kz1, wgt, acc, d);
            if (eta != T(0)) {
              const T cL = S.cd[jj - 1][ii];
              const int cnt = int(okR) + int(cell_ok(i, j - 1, k));
              acc += eta * (cR - cL);
              d += eta * T(cnt);
            }
            part += tile_finish<T, MODE>(fo[r][1], unsigned(k * pv) * E, j > 0 || unk_v0,
                                         acc * ih2, d * ih2, xf, bc[r][1], ry, omega, ry2);
          }
        }
        // ---- w-face (i, j, k): normal z
        {
          {
            const T xf = S.w[s][jj][ii];
            T acc = T(0), d = T(0);
            T kn0 = T(1), kn1 = T(1), kx0 = T(1), kx1 = T(1), ky0 = T(1), ky1 = T(1);
            if (VARMU) {
              kn0 = op.mu[cidx(G, i, j, max(k - 1, 0))];
              kn1 = op.mu[cidx(G, i, j, k)];
              kx0 = edge_mu<1>(op, i, j, k);
              kx1 = edge_mu<1>(op, i + 1, j, k);
              ky0 = edge_mu<0>(op, i, j, k);
              ky1 = edge_mu<0>(op, i, j + 1, k);
            }
            visc_axis<T>(xf, wp[r], S.w[s1][jj][ii], k > 0, true, false, false, kn0, kn1, T(1),
                         acc, d);
            const T wgt = (k == 0) ? T(0.5) : T(1);
            visc_axis<T>(xf, S.w[s][jj][ii - 1], S.w[s][jj][ii + 1], i > 0, i < nx - 1,
                         G.bc[0] == kDir, G.bc[1] == kDir, kx0, kx1, wgt, acc, d);
            visc_axis<T>(xf, S.w[s][jj - 1][ii], S.w[s][jj + 1][ii], j > 0, j < ny - 1,
                         G.bc[2] == kDir, G.bc[3] == kDir, ky0, ky1, wgt, acc, d);
            if (eta != T(0)) {
              const int cnt = int(okR) + int(cell_ok(i, j, k - 1));
              acc += eta * (cR - cdp[r]);
              d += eta * T(cnt);
            }
            part += tile_finish<T, MODE>(fo[r][1], unsigned(k * pw) * E + dw, k > 0 || unk_w0,
                                         acc * ih2, d * ih2, xf, bc[r][2], ry, omega, ry2);
          }
        }
        // upper boundary faces are Dirichlet faces: keep them zero
        if (i == nx - 1) buf_store(T(0), ry, fo[r][0] + E, unsigned(k * pu) * E);
        if (kAP) { if (i == nx - 1) buf_store(T(0), ry2, fo[r][0] + E, unsigned(k * pu) * E); }
        if (j == ny - 1) buf_store(T(0), ry, fo[r][1] + unsigned(nx) * E, unsigned(k * pv) * E);
        if (kAP) { if (j == ny - 1) buf_store(T(0), ry2, fo[r][1] + unsigned(nx) * E, unsigned(k * pv) * E); }
        if (k == nz - 1) buf_store(T(0), ry, fo[r][1], unsigned(nz * pw) * E + dw);
        if (kAP) { if (k == nz - 1) buf_store(T(0), ry2, fo[r][1], unsigned(nz * pw) * E + dw); }
        up[r] = S.u[s][jj][ii];
        vp[r] = S.v[s][jj][ii];
        wp[r] = S.w[s][jj][ii];
        cdp[r] = cR;
      }
    }
    fetch_b(min(k + 2, k1 - 1), bc);
    __syncthreads();
  };

  // Constant viscosity, one z-plane in two phases and two barriers: (A)
  // read every face neighbour, form the viscous part of M x and the
  // divergence of the own cells (written to LDS with the halo cells);
  // (B) add the grad-div term from the divergences of the neighbour cells
  // and finish.  The barrier before (A) of the next plane also orders the
  // divergence reads of (B) before their next writes.
  auto step_c = [&](int k, FRegs& F, BRegs& bc) {
    const int s = (k - k0) & 1, s1 = s ^ 1;
    store_plane(s1, k + 1, F);
    __syncthreads();
    fetch_plane(min(k + 3, k1), F);
    const bool pz = k == pk;
    const bool kbulk = k > 0 && k < nz - 1 && k != pk && k - 1 != pk;
    if (!kbulk) coef(k, false);  // uniform branch
    const T ww = k == 0 ? T(0.5) : T(1);
    // across the barrier: au / av = viscous part of M x + eta x own-cell
    // divergence for the u / v faces, and the face values (the next plane's
    // z neighbours); the w-face has both adjacent cells in this column and is
    // finished here
    T au[kRPT], av[kRPT];
#pragma unroll
    for (int r = 0; r < kRPT; ++r) {
      const int jj = ty + r * kTYT + 1, ii = tx + 1;
      const int i = i0 + tx, j = j0 + ty + r * kTYT;
      const T wu = i == 0 ? T(0.5) : T(1), wv = j == 0 ? T(0.5) : T(1);
      const T uC = S.u[s][jj][ii], uR = S.u[s][jj][ii + 1], uT = S.u[s1][jj][ii];
      const T vC = S.v[s][jj][ii], vN = S.v[s][jj + 1][ii], vT = S.v[s1][jj][ii];
      const T wC = S.w[s][jj][ii], wT = S.w[s1][jj][ii];
      const bool ok = i < nx && j < ny && !(pz && ((hbits >> (2 + r)) & 1u));
      const T cR = ok ? (uC - uR) + (vC - vN) + (wC - wT) : T(0);
      S.cd[jj][ii] = cR;
      au[r] = dv[r][0] * uC + eta * cR -
              ((S.u[s][jj][ii - 1] + uR) + wu * ((S.u[s][jj - 1][ii] + S.u[s][jj + 1][ii]) + (up[r] + uT)));
      av[r] = dv[r][1] * vC + eta * cR -
              ((S.v[s][jj - 1][ii] + vN) + wv * ((S.v[s][jj][ii - 1] + S.v[s][jj][ii + 1]) + (vp[r] + vT)));
      const T aw = dv[r][2] * wC + eta * (cR - cdp[r]) -
                   ((wp[r] + wT) + ww * ((S.w[s][jj][ii - 1] + S.w[s][jj][ii + 1]) +
                                         (S.w[s][jj - 1][ii] + S.w[s][jj + 1][ii])));
      if (i < nx && j < ny) {
        part += tile_out<T, MODE>(fo[r][1], unsigned(k * pw) * E + dw, k > 0 || unk_w0, aw * ih2,
                                  sc[r][2], wC, bc[r][2], ry, ry2);
        if (k == nz - 1) buf_store(T(0), ry, fo[r][1], unsigned(nz * pw) * E + dw);
        if (kAP) { if (k == nz - 1) buf_store(T(0), ry2, fo[r][1], unsigned(nz * pw) * E + dw); }
      }
      up[r] = uC;
      vp[r] = vC;
      wp[r] = wC;
      cdp[r] = cR;
    }
    if (threadIdx.x < kTX + 1 + kTY) {
      const int cj = hcj, ci = hci;
      const bool ok = (hbits & 1u) && !(pz && (hbits & 2u));
      const T v = (S.u[s][cj][ci] - S.u[s][cj][ci + 1]) + (S.v[s][cj][ci] - S.v[s][cj + 1][ci]) +
                  (S.w[s][cj][ci] - S.w[s1][cj][ci]);
      S.cd[cj][ci] = ok ? v : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRPT; ++r) {
      const int jj = ty + r * kTYT + 1, ii = tx + 1;
      const int i = i0 + tx, j = j0 + ty + r * kTYT;
      if (i < nx && j < ny) {
        part += tile_out<T, MODE>(fo[r][0], unsigned(k * pu) * E, i > 0 || unk_u0,
                                  (au[r] - eta * S.cd[jj][ii - 1]) * ih2, sc[r][0], up[r],
                                  bc[r][0], ry, ry2);
        part += tile_out<T, MODE>(fo[r][1], unsigned(k * pv) * E, j > 0 || unk_v0,
                                  (av[r] - eta * S.cd[jj - 1][ii]) * ih2, sc[r][1], vp[r],
                                  bc[r][1], ry, ry2);
        // upper boundary faces are Dirichlet faces: keep them zero
        if (i == nx - 1) buf_store(T(0), ry, fo[r][0] + E, unsigned(k * pu) * E);
        if (kAP) { if (i == nx - 1) buf_store(T(0), ry2, fo[r][0] + E, unsigned(k * pu) * E); }
        if (j == ny - 1) buf_store(T(0), ry, fo[r][1] + unsigned(nx) * E, unsigned(k * pv) * E);
        if (kAP) { if (j == ny - 1) buf_store(T(0), ry2, fo[r][1] + unsigned(nx) * E, unsigned(k * pv) * E); }
      }
    }
    if (!kbulk) coef(0, true);
    fetch_b(min(k + 2, k1 - 1), bc);
  };
  if constexpr (VARMU) {
    for (int k = k0; k < k1; k += 2) {
      step(k, FA, bA);
      if (k + 1 < k1) step(k + 1, FB, bB);
    }
  } else {
    for (int k = k0; k < k1; k += 2) {
      step_c(k, FA, bA);
      if (k + 1 < k1) step_c(k + 1, FB, bB);
    }
  }
  constexpr bool kRed = MODE == kApplyDot || MODE == kJacobiDot || MODE == kDinvM ||
                        MODE == kResidDot || MODE == kApplyDotP;
  if (kRed) {
    __shared__ double sh[256 / 64];
    double t = block_sum<256>(part, sh);
    if (threadIdx.x == 0)
      partial[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = t;
  }
}

}  // namespace gkb
