// Host runtime and C-ABI of the GKB solver (see include/gkb.h).
//
// One gkb_solve runs generalized Golub-Kahan bidiagonalization (Section 2):
// the change of variables that leaves a zero first right-hand side, then
// columns of the bidiagonal B from the relations A Q = M V B and
// A^T V = N Q B^T, each needing one inner solve with M = W + eta A A^T,
// turned into the Craig-variant iterates (u, p) and stopped by the delayed
// lower bound of Section 2.2.  Optional around it: defect correction in FP64
// (mixed precision), or an outer FGMRES that uses the GKB run as its
// preconditioner (Section 3).  The scalars of the outer recurrence live on
// the host in FP64; every vector operation is a HIP kernel.  The inner
// solves (the dominant cost) are PCG, flexible CG or FGMRES iterations whose
// scalars stay on the device; chunks of iterations are captured in HIP
// graphs and replayed until the device-side convergence flag is set
// (iterations after convergence are no-ops).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gkb.h"
#include "kernels.hpp"
#include "cnn.hpp"
#include "learned.hpp"
#include "tile3d.hpp"
#include "hybrid.hpp"
#include "fgmres.hpp"
#include "csr.hpp"

using namespace gkb;

#define HIPCK(expr)                                                     \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) {                                             \
      std::fprintf(stderr, "gkb: HIP error %s at %s:%d\n",              \
                   hipGetErrorString(e_), __FILE__, __LINE__);          \
      return GKB_EHIP;                                                  \
    }                                                                   \
  } while (0)

#define CK(expr)                  \
  do {                            \
    int rc_ = (expr);             \
    if (rc_ < 0) return rc_;      \
  } while (0)

namespace {

constexpr int kMaxLevels = 16;
constexpr int kSlots = 6;
constexpr int kMaxRestart = kGmMaxRestart;  // inner FGMRES Krylov vectors
constexpr int kMaxOuterRestart = 32;  // outer FGMRES (GKB as preconditioner)

int vec_blocks(int n) { return std::max(1, std::min((n + 1023) / 1024, 4096)); }

struct FaceLaunch {
  dim3 grid;
  int kz = 1, zchunks = 1;
  int nparts = 0;   // partials written by face_op's reduction modes
  int gparts = 0;   // partials of kernels launched on the generic grid
  bool tiled = false;  // LDS-tiled 3D kernel for the stencil modes
  dim3 tgrid;
  int tz = 8;
};

FaceLaunch face_launch(const Grid& g, int kz, int stencil = 0) {
  FaceLaunch L;
  int maxplane = 0;
  for (int c = 0; c < g.dim; ++c) maxplane = std::max(maxplane, g.ext[c][0] * g.ext[c][1]);
  L.kz = kz;
  L.zchunks = (g.nze + kz - 1) / kz;
  L.grid = dim3((maxplane + kBlock - 1) / kBlock, 1, g.dim * L.zchunks);
  L.nparts = L.grid.x * L.grid.z;
  L.gparts = L.nparts;
  // the tiled kernel covers the lower faces of every cell: the upper faces
  // must be Dirichlet (zero) faces
  const bool upper_dir = g.bc[1] == kDir && g.bc[3] == kDir && g.bc[5] == kDir;
  // (32-bit buffer offsets: face arrays below 2 GiB in FP64)
  if (stencil == 0 && g.dim == 3 && upper_dir && (long)g.m_full * 8 < (1L << 31)) {
    L.tiled = true;
    const int tx = (g.n[0] + kTX - 1) / kTX, ty = (g.n[1] + kTY - 1) / kTY;
    // z-planes per block: keep >= ~512 blocks in flight; more planes per
    // block amortise the z-halo and the block set-up but starve small grids
    // (128^3: 8 planes, 1024 blocks, where 2, 4 and 16 were slower; 64^3: 2
    // planes, 512 blocks, 1-3 % faster MG-PCG iterations than 1 or 4)
    const int tz = std::max(1, std::min(8, tx * ty * g.n[2] / 512));
    L.tz = std::min(tz, g.n[2]);
    L.tgrid = dim3(tx, ty, (g.n[2] + L.tz - 1) / L.tz);
    L.nparts = L.tgrid.x * L.tgrid.y * L.tgrid.z;
  }
  return L;
}

dim3 cell_grid(const Grid& g) {
  return dim3((g.n[0] * g.n[1] + kBlock - 1) / kBlock, 1, g.n[2]);
}
int cell_parts(const Grid& g) { return cell_grid(g).x * g.n[2]; }

dim3 transfer_grid(const Grid& g) {
  int maxplane = 0;
  for (int c = 0; c < g.dim; ++c) maxplane = std::max(maxplane, g.ext[c][0] * g.ext[c][1]);
  return dim3((maxplane + kBlock - 1) / kBlock, 1, g.dim * g.nze);
}

template <typename T>
struct DevArr {
  T* p = nullptr;
};

struct Alloc {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  size_t cap = 0;
  hipStream_t s = nullptr;  // the context stream: zero fills are ordered on it
  int get(void** out, size_t b) {
    if (cap && bytes + b > cap) return GKB_ENOMEM;
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(b, 256)) != hipSuccess) return GKB_ENOMEM;
    ptrs.push_back(q);
    // zero-filled: faces that no kernel writes (Dirichlet faces) read as 0
    if (hipMemsetAsync(q, 0, std::max<size_t>(b, 256), s) != hipSuccess) return GKB_EHIP;
    bytes += b;
    *out = q;
    return GKB_OK;
  }
  template <typename T>
  int arr(T** out, size_t n) {
    return get(reinterpret_cast<void**>(out), n * sizeof(T));
  }
  void release() {
    for (void* q : ptrs) (void)hipFree(q);
    ptrs.clear();
    bytes = 0;
  }
};

// coefficient arrays of one level in one precision
template <typename T>
struct Coef {
  T* mu = nullptr;
  T* mue[3] = {nullptr, nullptr, nullptr};
};

template <typename T>
struct Level {
  Grid g;
  Op<T> op;
  T *b = nullptr, *x = nullptr, *t = nullptr, *rb = nullptr;
  double omega = 0.8;
  FaceLaunch fl;
  // hybrid smoother: 1/diag(C^T W C) on the edges (nullptr: Jacobi only)
  T* edinv = nullptr;
  // 1/diag(M_l) on the coarse levels that smooth: the restriction into the
  // level writes its first sweep from a zero guess in the same pass
  T* dinv = nullptr;
  double omega_e = 0.0;
};

template <typename T>
struct Inner {
  bool ready = false;
  std::vector<Level<T>> lv;
  T *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *dinv = nullptr;
  T* p2 = nullptr;     // second direction buffer of the fused direction update
  T *rprev = nullptr;  // flexible CG
  PcgState* st = nullptr;
  // captured chunks of iterations: PCG (Jacobi or MG preconditioner) and
  // flexible CG with the network, kept apart because the learned mode falls
  // back to plain MG-PCG
  hipGraphExec_t graph = nullptr;
  int graph_len = 0;
  int graph_mode = -1;
  hipGraphExec_t graph_fcg = nullptr;
  int graph_fcg_len = 0;
  // inner FGMRES: basis V (restart + 1 vectors) and preconditioned vectors Z
  // (restart), FP64 Hessenberg state, the cycle flag and the dot partials;
  // one restart cycle is one captured graph
  T *gm_V = nullptr, *gm_Z = nullptr;
  FgmState* gm_fs = nullptr;
  PcgState* gm_cyc = nullptr;
  double* gm_part = nullptr;
  hipGraphExec_t graph_gm = nullptr;
  bool graph_gm_learned = false;  // the captured cycle applies the network
};

// the learned preconditioner z = V(r) + theta c applied to r_in
// (learned_impl.hpp)
template <typename T>
void learned_apply(gkb_ctx* c, Inner<T>& in, const T* r_in, T* z_out, const PcgState* st_dot,
                   PcgState* st);

}  // namespace

struct gkb_ctx {
  Grid g;
  double eta = 0.0;
  gkb_options opt;
  hipStream_t us = nullptr;  // caller stream (may be null)
  hipStream_t cs = nullptr;  // own non-blocking stream
  hipEvent_t ev = nullptr;
  bool varmu = false;
  bool smooth_transfer = false;  // SMOOTH multigrid transfers (else DIV)
  Alloc mem;
  int L = 1;
  std::vector<Grid> grids;
  std::vector<Coef<double>> coef64;
  std::vector<Coef<float>> coef32;
  std::vector<double> omega;
  std::vector<double> omega_e;               // edge-sweep weights (hybrid)
  std::vector<std::vector<double>> edinv_h;  // 1/diag(C^T W C) per level (hybrid)
  Op<double> op64;  // finest FP64 M
  Op<float> op32;
  double* Minv = nullptr;
  int mc = 0;
  Inner<double> in64;
  Inner<float> in32;
  // GKB vectors
  double *ghat = nullptr, *w0 = nullptr, *u = nullptr, *v = nullptr, *Mv = nullptr, *s = nullptr,
         *y = nullptr, *f = nullptr, *rw = nullptr, *dw = nullptr;
  double *wbest = nullptr, *pbest = nullptr;  // best defect-correction iterate
  // GKB as the preconditioner of an outer FGMRES: basis V (outer_restart + 1)
  // and preconditioned vectors Z (outer_restart), each a (faces | cells)
  // pair of m_full + n_cells doubles, and a zero pair
  double *ov = nullptr, *oz = nullptr, *ozero = nullptr;
  double *b = nullptr, *q = nullptr, *d = nullptr, *t = nullptr, *rr = nullptr, *dp = nullptr;
  double* part[kSlots] = {nullptr};
  int maxparts = 0;
  double* dscal = nullptr;
  double* hbuf = nullptr;  // pinned host
  FaceLaunch fl0;
  gkb_stats_t stats;
  Learned* learned = nullptr;
  gkb_cnn* owned_net = nullptr;  // network loaded from opt.cnn_weights
  // assembled (CSR) system instead of the MAC grid: operators, A'^T x
  // temporaries per precision, central-scaling state and scaled right-hand
  // sides
  bool csr = false;
  bool csr_scaled = false;
  CsrOps<double> csr64;
  CsrOps<float> csr32;
  double* csr_t64 = nullptr;
  float* csr_t32 = nullptr;
  double *csr_gs = nullptr, *csr_rs = nullptr;
};

namespace {

// ------------------------------------------------------------ launches

template <typename T>
const CsrOps<T>& csr_of(const gkb_ctx* c);
template <>
const CsrOps<double>& csr_of<double>(const gkb_ctx* c) { return c->csr64; }
template <>
const CsrOps<float>& csr_of<float>(const gkb_ctx* c) { return c->csr32; }
template <typename T>
T* csr_tmp(gkb_ctx* c);
template <>
double* csr_tmp<double>(gkb_ctx* c) { return c->csr_t64; }
template <>
float* csr_tmp<float>(gkb_ctx* c) { return c->csr_t32; }

// the M-apply modes on an assembled system (t = A'^T x first)
template <typename T, int MODE>
void csr_face_op(gkb_ctx* c, T eta, const T* x, const T* b, T* y, double* partial,
                 const PcgState* st) {
  const CsrOps<T>& o = csr_of<T>(c);
  hipStream_t s = c->cs;
  if constexpr (MODE == kApply || MODE == kApplyDot || MODE == kResid || MODE == kResidDot ||
                MODE == kDiag) {
    T* t = csr_tmp<T>(c);
    if (MODE != kDiag && eta != T(0)) k_csr_at<T><<<vec_blocks(o.n), kBlock, 0, s>>>(o, x, t, st);
    k_csr_m<T, MODE><<<vec_blocks(o.m), kBlock, 0, s>>>(o, eta, x, t, b, y, partial, st);
  }
}

// partials written by the A^T kernel (div_axpy)
int div_parts(const gkb_ctx* c) {
  return c->csr ? vec_blocks(c->g.n_cells) : cell_parts(c->g);
}

// ec / Gc: coarse correction and coarse grid of kJacobiP (unused otherwise)
template <typename T, int MODE>
void face_op(gkb_ctx* c, const Op<T>& op, const FaceLaunch& fl, const T* x, const T* b, T* y,
             T omega, double* partial, const PcgState* st, const T* ec = nullptr,
             const Grid* Gc = nullptr, T* y2 = nullptr) {
  if (c->csr) {
    csr_face_op<T, MODE>(c, op.eta, x, b, y, partial, st);
    return;
  }
  const bool vm = op.mu != nullptr;
  const int kz = fl.kz, zc = fl.zchunks;
  hipStream_t s = c->cs;
  const Grid gc = Gc ? *Gc : op.g;
  if constexpr (MODE == kJacobiZ) {
    // tiled grids with constant viscosity only (the caller checks)
    const bool fine = op.g.m_full == c->g.m_full;
    if (fine) k_tile3d<T, false, MODE, true><<<fl.tgrid, 256, 0, s>>>(op, x, b, y, omega, fl.tz, partial, st, ec, gc, y2);
    else k_tile3d<T, false, MODE, false><<<fl.tgrid, 256, 0, s>>>(op, x, b, y, omega, fl.tz, partial, st, ec, gc, y2);
    return;
  } else {
    if (fl.tiled && MODE != kJacobi0 && MODE != kDiag) {
      const bool fine = op.g.m_full == c->g.m_full;
      if (vm) {
        if (fine) k_tile3d<T, true, MODE, true><<<fl.tgrid, 256, 0, s>>>(op, x, b, y, omega, fl.tz, partial, st, ec, gc, y2);
        else k_tile3d<T, true, MODE, false><<<fl.tgrid, 256, 0, s>>>(op, x, b, y, omega, fl.tz, partial, st, ec, gc, y2);
      } else {
        if (fine) k_tile3d<T, false, MODE, true><<<fl.tgrid, 256, 0, s>>>(op, x, b, y, omega, fl.tz, partial, st, ec, gc, y2);
        else k_tile3d<T, false, MODE, false><<<fl.tgrid, 256, 0, s>>>(op, x, b, y, omega, fl.tz, partial, st, ec, gc, y2);
      }
      return;
    }
    if constexpr (MODE == kJacobiP || MODE == kApplyDotP) return;  // tiled only (the caller checks)
    if (op.g.dim == 2) {
      if (vm) k_face_op<T, 2, true, MODE><<<fl.grid, kBlock, 0, s>>>(op, x, b, y, omega, kz, zc, partial, st);
      else k_face_op<T, 2, false, MODE><<<fl.grid, kBlock, 0, s>>>(op, x, b, y, omega, kz, zc, partial, st);
    } else {
      if (vm) k_face_op<T, 3, true, MODE><<<fl.grid, kBlock, 0, s>>>(op, x, b, y, omega, kz, zc, partial, st);
      else k_face_op<T, 3, false, MODE><<<fl.grid, kBlock, 0, s>>>(op, x, b, y, omega, kz, zc, partial, st);
    }
  }
}

void grad_axpy(gkb_ctx* c, const double* q, const double* yv, double s1, double s2, double* out) {
  if (c->csr) {
    k_csr_grad<<<vec_blocks(c->g.m_full), kBlock, 0, c->cs>>>(c->csr64, q, yv, s1, s2, out);
    return;
  }
  const FaceLaunch& fl = c->fl0;
  if (c->g.dim == 2)
    k_grad_axpy<2><<<fl.grid, kBlock, 0, c->cs>>>(c->g, q, yv, s1, s2, out, fl.kz, fl.zchunks);
  else
    k_grad_axpy<3><<<fl.grid, kBlock, 0, c->cs>>>(c->g, q, yv, s1, s2, out, fl.kz, fl.zchunks);
}

template <typename T>
void div_axpy(gkb_ctx* c, const Grid& g, const T* x, const T* z, double s1, double s2, T* t,
              double* partial, double* zz) {
  if (c->csr) {
    k_csr_div<T><<<vec_blocks(g.n_cells), kBlock, 0, c->cs>>>(csr_of<T>(c), x, z, s1, s2, t,
                                                               partial, zz);
    return;
  }
  if (g.dim == 2)
    k_div_axpy<T, 2><<<cell_grid(g), kBlock, 0, c->cs>>>(g, x, z, s1, s2, t, partial, zz);
  else
    k_div_axpy<T, 3><<<cell_grid(g), kBlock, 0, c->cs>>>(g, x, z, s1, s2, t, partial, zz);
}

int host_sum(gkb_ctx* c, const double* partial, int n, double* out) {
  k_sum_partials<<<1, kFinal, 0, c->cs>>>(partial, n, c->dscal);
  HIPCK(hipMemcpyAsync(c->hbuf, c->dscal, sizeof(double), hipMemcpyDeviceToHost, c->cs));
  HIPCK(hipStreamSynchronize(c->cs));
  *out = c->hbuf[0];
  return GKB_OK;
}

// ---------------------------------------------------------- multigrid

// x += C omega_e D_e^-1 C^T (b - M x): the edge half of the hybrid smoother
template <typename T>
void edge_step(gkb_ctx* c, Level<T>& L, const T* b, T* x, const PcgState* st) {
  hipStream_t s = c->cs;
  face_op<T, kResid>(c, L.op, L.fl, x, b, L.rb, T(0), nullptr, st);
  const dim3 cg = cell_grid(L.g);
  if (L.g.dim == 2) k_edge_smooth<T, 2><<<cg, kBlock, 0, s>>>(L.g, L.rb, L.edinv, T(L.omega_e), x, st);
  else k_edge_smooth<T, 3><<<cg, kBlock, 0, s>>>(L.g, L.rb, L.edinv, T(L.omega_e), x, st);
}

// first smoothing sweep from a zero guess, x = omega D^-1 b, from 1 / D
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi_first(int n, T omega, const T* __restrict__ dinv,
                                                         const T* __restrict__ b,
                                                         T* __restrict__ x, const PcgState* st) {
  if (st && st->done) return;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    x[i] = omega * dinv[i] * b[i];
}

// first_done: the first pre-smoothing sweep from a zero guess is already in
// its output buffer (written by the restriction into this level)
template <typename T>
void vcycle(gkb_ctx* c, Inner<T>& in, int l, const T* b, T* x, double* dot_partial,
            const PcgState* st, bool first_done = false) {
  Level<T>& L = in.lv[l];
  hipStream_t s = c->cs;
  if (l == c->L - 1) {
    const int m = L.g.m_full;
    k_coarse_gemv<T><<<(m + 3) / 4, kBlock, m * sizeof(double), s>>>(m, c->Minv, b, x, st);
    if (dot_partial) {
      k_dot<T><<<vec_blocks(m), kBlock, 0, s>>>(m, b, x, dot_partial);
    }
    return;
  }
  const int n1 = c->opt.nu_pre, n2 = c->opt.nu_post, tot = n1 + n2;
  const T om = T(L.omega);
  const bool hybrid = L.edinv != nullptr;
  // sweep k writes x when (tot - k) is even, else t
  auto dst = [&](int k) { return ((tot - k) % 2 == 0) ? x : L.t; };
  const T* cur = nullptr;
  int k = 0;
  if (n1 > 0) {
    int i = 1;
    ++k;
    // the first two sweeps from a zero guess in one pass (tiled grids,
    // constant viscosity, weighted-Jacobi smoother)
    const bool two = !first_done && n1 >= 2 && !hybrid && L.fl.tiled && L.op.mu == nullptr;
    if (two) {
      ++k;
      ++i;
      face_op<T, kJacobiZ>(c, L.op, L.fl, b, b, dst(k), om, nullptr, st);
      cur = dst(k);
    } else {
      T* o = dst(k);
      // x = omega D^-1 b from the stored 1 / D (finest level: the Jacobi
      // preconditioner's), a plain stream instead of the stencil pass
      // that forms D face by face (variable viscosity reads every
      // coefficient array for it)
      const T* dv = (l == 0) ? in.dinv : L.dinv;
      if (!first_done) {
        if (dv)
          k_jacobi_first<T><<<vec_blocks(L.g.m_full), kBlock, 0, s>>>(L.g.m_full, om, dv, b, o, st);
        else
          face_op<T, kJacobi0>(c, L.op, L.fl, nullptr, b, o, om, nullptr, st);
      }
      if (hybrid) edge_step<T>(c, L, b, o, st);
      cur = o;
    }
    for (; i < n1; ++i) {
      ++k;
      T* o2 = dst(k);
      face_op<T, kJacobi>(c, L.op, L.fl, cur, b, o2, om, nullptr, st);
      if (hybrid) edge_step<T>(c, L, b, o2, st);
      cur = o2;
    }
  }
  Level<T>& Lc = in.lv[l + 1];
  const dim3 tg = transfer_grid(Lc.g);
  // the coarse level's first sweep (x = omega D^-1 b) goes where its V-cycle
  // puts the first pre-smoothing result
  T* x0c = (n1 > 0 && Lc.dinv) ? (((tot - 1) % 2 == 0) ? Lc.x : Lc.t) : nullptr;
  const T omc = T(Lc.omega);
  const T* rsrc = cur ? L.rb : b;
  if (cur) face_op<T, kResid>(c, L.op, L.fl, cur, b, L.rb, T(0), nullptr, st);
  const bool sm = c->smooth_transfer;
  if (L.g.dim == 2) {
    if (sm) k_restrict<T, 2, true><<<tg, kBlock, 0, s>>>(L.g, Lc.g, rsrc, Lc.b, st, Lc.dinv, omc, x0c);
    else k_restrict<T, 2, false><<<tg, kBlock, 0, s>>>(L.g, Lc.g, rsrc, Lc.b, st, Lc.dinv, omc, x0c);
  } else {
    // fine v, w pairs (2i, 2i+1) aligned: even x extent and array offsets
    // (FP32 only: the 16-byte FP64 pairs measured slower than two loads)
    const int pair = sizeof(T) == 4 && L.g.n[0] % 2 == 0 && L.g.off[1] % 2 == 0 &&
                     L.g.off[2] % 2 == 0;
    if (sm) k_restrict<T, 3, true><<<tg, kBlock, 0, s>>>(L.g, Lc.g, rsrc, Lc.b, st, Lc.dinv, omc, x0c);
    else k_restrict<T, 3, false><<<tg, kBlock, 0, s>>>(L.g, Lc.g, rsrc, Lc.b, st, Lc.dinv, omc, x0c,
                                                        pair);
  }
  vcycle<T>(c, in, l + 1, Lc.b, Lc.x, nullptr, st, x0c != nullptr);
  // prolongate into the current iterate (or into a zeroed x when no pre-smoothing)
  T* it = const_cast<T*>(cur);
  if (!it) {
    it = (n2 % 2 == 0) ? x : L.t;
    k_fill<T><<<vec_blocks(L.g.m_full), kBlock, 0, s>>>(L.g.m_full, T(0), it);
  }
  // the coarse-grid correction is added while the first post-smoothing sweep
  // stages its input (tiled grids, weighted-Jacobi smoother, divergence-
  // compatible transfers, that sweep not the one that forms the dot product)
  const bool pro = cur && n2 >= 1 && !hybrid && !sm && L.fl.tiled && !(n2 == 1 && dot_partial);
  int i0 = 0;
  if (pro) {
    ++k;
    T* o = (it == x) ? L.t : x;
    face_op<T, kJacobiP>(c, L.op, L.fl, it, b, o, om, nullptr, st, Lc.x, &Lc.g);
    cur = o;
    i0 = 1;
  } else {
    const dim3 fg = transfer_grid(L.g);
    if (L.g.dim == 2) {
      if (sm) k_prolong_add<T, 2, true><<<fg, kBlock, 0, s>>>(L.g, Lc.g, Lc.x, it, st);
      else k_prolong_add<T, 2, false><<<fg, kBlock, 0, s>>>(L.g, Lc.g, Lc.x, it, st);
    } else {
      if (sm) k_prolong_add<T, 3, true><<<fg, kBlock, 0, s>>>(L.g, Lc.g, Lc.x, it, st);
      else k_prolong_add<T, 3, false><<<fg, kBlock, 0, s>>>(L.g, Lc.g, Lc.x, it, st);
    }
    cur = it;
  }
  for (int i = i0; i < n2; ++i) {
    ++k;
    T* o = (cur == x) ? L.t : x;
    const bool last = (i == n2 - 1);
    if (hybrid) edge_step<T>(c, L, b, const_cast<T*>(cur), st);
    if (last && dot_partial)
      face_op<T, kJacobiDot>(c, L.op, L.fl, cur, b, o, om, dot_partial, st);
    else
      face_op<T, kJacobi>(c, L.op, L.fl, cur, b, o, om, nullptr, st);
    cur = o;
  }
  if (cur != x) {
    k_cast<T, T><<<vec_blocks(L.g.m_full), kBlock, 0, s>>>(L.g.m_full, cur, x);
  }
  if (n2 == 0 && dot_partial) {
    k_dot<T><<<vec_blocks(L.g.m_full), kBlock, 0, s>>>(L.g.m_full, b, x, dot_partial);
  }
}

template <typename T>
int vcycle_parts(gkb_ctx* c, Inner<T>& in) {
  if (c->L == 1) return vec_blocks(in.lv[0].g.m_full);
  if (c->opt.nu_post == 0) return vec_blocks(in.lv[0].g.m_full);
  return in.lv[0].fl.nparts;
}

// -------------------------------------------------------------- PCG

template <typename T>
Inner<T>& inner_of(gkb_ctx* c);
template <>
Inner<double>& inner_of<double>(gkb_ctx* c) { return c->in64; }
template <>
Inner<float>& inner_of<float>(gkb_ctx* c) { return c->in32; }

template <typename T>
const Op<T>& op_of(gkb_ctx* c);
template <>
const Op<double>& op_of<double>(gkb_ctx* c) { return c->op64; }
template <>
const Op<float>& op_of<float>(gkb_ctx* c) { return c->op32; }

template <typename T>
int pcg_iterations(gkb_ctx* c, Inner<T>& in, int count) {
  const Level<T>& L0 = in.lv[0];
  const int n = L0.g.m_full, vb = vec_blocks(n);
  hipStream_t s = c->cs;
  const bool jac = c->opt.inner == GKB_INNER_JACOBI;
  // MG-PCG on a tiled finest grid: the direction update p = z + beta p is
  // formed while the product q = M p stages its input, alternating between
  // in.p and in.p2 (an even count of iterations ends in in.p; the first
  // iteration of a solve has beta = 0 and in.p = z).  FP32 only: the FP64
  // kernel needs 152 VGPRs, one wave per SIMD fewer than the plain product,
  // and measured 2 % slower per iteration
  const bool fused = sizeof(T) == 4 && !jac && L0.fl.tiled && in.p2 && count % 2 == 0;
  for (int it = 0; it < count; ++it) {
    T* pd = in.p;  // direction of this iteration
    if (fused) {
      T* pold = (it % 2 == 0) ? in.p : in.p2;
      pd = (it % 2 == 0) ? in.p2 : in.p;
      face_op<T, kApplyDotP>(c, L0.op, L0.fl, in.z, pold, in.q, T(0), c->part[0], in.st,
                             nullptr, nullptr, pd);
    } else {
      face_op<T, kApplyDot>(c, L0.op, L0.fl, in.p, nullptr, in.q, T(0), c->part[0], in.st);
    }
    k_pcg_alpha<<<1, kFinal, 0, s>>>(in.st, c->part[0], L0.fl.nparts);
    if (jac) {
      k_pcg_xr<T><<<vb, kBlock, 0, s>>>(n, in.st, pd, in.q, in.x, in.r, in.dinv, in.z,
                                        c->part[1], c->part[2]);
      k_pcg_check<<<1, kFinal, 0, s>>>(in.st, c->part[1], vb, c->part[2], vb);
    } else {
      k_pcg_xr<T><<<vb, kBlock, 0, s>>>(n, in.st, pd, in.q, in.x, in.r, nullptr, nullptr,
                                        c->part[1], nullptr);
      k_pcg_check<<<1, kFinal, 0, s>>>(in.st, c->part[1], vb, nullptr, 0);
      vcycle<T>(c, in, 0, in.r, in.z, c->part[2], in.st);
      k_pcg_beta<<<1, kFinal, 0, s>>>(in.st, c->part[2], vcycle_parts<T>(c, in));
    }
    if (!fused) k_pcg_p<T><<<vb, kBlock, 0, s>>>(n, in.st, in.z, in.p);
  }
  return GKB_OK;
}

template <typename T>
int ensure_graph(gkb_ctx* c, Inner<T>& in, int count) {
  // the PCG iteration depends only on the preconditioner (Jacobi or V-cycle)
  const int key = c->opt.inner == GKB_INNER_JACOBI ? GKB_INNER_JACOBI : GKB_INNER_MG;
  if (in.graph && in.graph_len == count && in.graph_mode == key) return GKB_OK;
  if (in.graph) {
    (void)hipGraphExecDestroy(in.graph);
    in.graph = nullptr;
  }
  hipGraph_t gr;
  HIPCK(hipStreamBeginCapture(c->cs, hipStreamCaptureModeThreadLocal));
  const int prc = pcg_iterations<T>(c, in, count);
  const hipError_t ce = hipStreamEndCapture(c->cs, &gr);
  if (prc < 0) {
    if (ce == hipSuccess) (void)hipGraphDestroy(gr);
    return prc;
  }
  HIPCK(ce);
  const hipError_t ie = hipGraphInstantiate(&in.graph, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  HIPCK(ie);
  in.graph_len = count;
  in.graph_mode = key;
  return GKB_OK;
}

// One restart cycle of the inner FGMRES (fgmres.hpp): Arnoldi steps
// j = 0 .. restart-1 with z_j = P(v_j) (Jacobi or one V-cycle) and
// w = M z_j orthogonalised by two classical Gram-Schmidt passes, then
// x += Z y, and the next cycle's start from the true residual r = f - M x
// (f in in.rprev).  Every kernel skips once its flag is set, so the launch
// sequence is fixed and is captured as one graph.
template <typename T>
void fgmres_cycle(gkb_ctx* c, Inner<T>& in) {
  const Level<T>& L0 = in.lv[0];
  const int n = L0.g.m_full, vb = vec_blocks(n);
  const int R = c->opt.fgmres_restart;
  const long ld = n;
  hipStream_t s = c->cs;
  const bool jac = c->opt.inner == GKB_INNER_JACOBI;
  const bool learned = c->opt.inner == GKB_INNER_LEARNED && learned_has_net(c->learned);
  for (int j = 0; j < R; ++j) {
    T* vj = in.gm_V + j * ld;
    T* zj = in.gm_Z + j * ld;
    T* w = in.gm_V + (j + 1) * ld;
    if (jac) k_gm_jacobi<T><<<vb, kBlock, 0, s>>>(n, in.gm_cyc, in.dinv, vj, zj);
    else if (learned) learned_apply<T>(c, in, vj, zj, in.gm_cyc, in.gm_cyc);
    else vcycle<T>(c, in, 0, vj, zj, nullptr, in.gm_cyc);
    face_op<T, kApply>(c, L0.op, L0.fl, zj, nullptr, w, T(0), nullptr, in.gm_cyc);
    const int nv = j + 1;
    const dim3 dg(vb, (nv + kGmChunk - 1) / kGmChunk);
    for (int pass = 0; pass < 2; ++pass) {
      k_gm_mdot<T><<<dg, kBlock, 0, s>>>(n, in.gm_cyc, in.gm_V, ld, nv, w, in.gm_part);
      k_gm_hsum<<<1, kFinal, 0, s>>>(in.gm_cyc, in.gm_fs, in.gm_part, vb, nv, j, pass);
      k_gm_maxpy<T><<<vb, kBlock, 0, s>>>(n, in.gm_cyc, in.gm_fs, in.gm_V, ld, nv, w, c->part[0]);
    }
    k_gm_arnoldi_end<<<1, kFinal, 0, s>>>(in.st, in.gm_cyc, in.gm_fs, c->part[0], vb, j,
                                          j == R - 1 ? 1 : 0);
    k_gm_scale<T><<<vb, kBlock, 0, s>>>(n, in.gm_cyc, in.gm_fs, j, w);
  }
  k_gm_solve_y<<<1, 64, 0, s>>>(in.st, in.gm_fs);
  k_gm_update_x<T><<<vb, kBlock, 0, s>>>(n, in.st, in.gm_fs, in.gm_Z, ld, in.x);
  k_gm_cycle_end<<<1, 64, 0, s>>>(in.st, in.gm_fs);
  face_op<T, kResidDot>(c, L0.op, L0.fl, in.x, in.rprev, in.r, T(0), c->part[1], in.st);
  k_gm_start<<<1, kFinal, 0, s>>>(in.st, in.gm_cyc, in.gm_fs, c->part[1], L0.fl.nparts, 0.0, 0, 0,
                                  sizeof(T) == 4 ? 1 : 0);
  k_gm_v0<T><<<vb, kBlock, 0, s>>>(n, in.st, in.gm_fs, in.r, in.gm_V);
}

int learned_prepare(gkb_ctx* c);

template <typename T>
int fgmres_solve(gkb_ctx* c, const double* f, double* x_out, double tol, int* iters) {
  Inner<T>& in = inner_of<T>(c);
  const int n = in.lv[0].g.m_full, vb = vec_blocks(n);
  hipStream_t s = c->cs;
  // the learned preconditioner (FGMRES takes any preconditioner, also one
  // that changes from step to step): network buffers and BF16 weights ready
  // before the cycle is captured or replayed
  const bool learned = c->opt.inner == GKB_INNER_LEARNED && learned_has_net(c->learned);
  if (learned) CK(learned_prepare(c));
  if (in.graph_gm && in.graph_gm_learned != learned) {
    (void)hipGraphExecDestroy(in.graph_gm);
    in.graph_gm = nullptr;
  }
  k_pcg_init<double, T><<<vb, kBlock, 0, s>>>(n, f, in.x, in.r, c->part[3]);
  k_cast<T, T><<<vb, kBlock, 0, s>>>(n, in.r, in.rprev);  // f in working precision
  k_gm_start<<<1, kFinal, 0, s>>>(in.st, in.gm_cyc, in.gm_fs, c->part[3], vb, tol,
                                  c->opt.inner_maxit, 1, 0);
  k_gm_v0<T><<<vb, kBlock, 0, s>>>(n, in.st, in.gm_fs, in.r, in.gm_V);
  if (c->opt.use_graphs && !in.graph_gm) {
    hipGraph_t gr;
    HIPCK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    fgmres_cycle<T>(c, in);
    HIPCK(hipStreamEndCapture(s, &gr));
    const hipError_t ie = hipGraphInstantiate(&in.graph_gm, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    HIPCK(ie);
    in.graph_gm_learned = learned;
  }
  PcgState hs;
  // every cycle takes at least one Arnoldi step, so inner_maxit bounds the
  // number of cycles
  for (long cyc = 0; cyc <= (long)c->opt.inner_maxit; ++cyc) {
    if (c->opt.use_graphs) HIPCK(hipGraphLaunch(in.graph_gm, s));
    else fgmres_cycle<T>(c, in);
    HIPCK(hipMemcpyAsync(c->hbuf, in.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    std::memcpy(&hs, c->hbuf, sizeof(PcgState));
    if (hs.done) break;
  }
  k_cast<T, double><<<vb, kBlock, 0, s>>>(n, in.x, x_out);
  if (iters) *iters = hs.it;
  c->stats.inner_iterations += hs.it;
  c->stats.inner_solves += 1;
  if (learned) c->stats.learned_solves += 1;
  if (hs.nonfinite) return GKB_ENAN;
  if (!hs.done || hs.status == -5) return GKB_EINNER;
  return GKB_OK;
}

// x_out = M^-1 f (FP64 in and out; T = working precision of the inner solve)
template <typename T>
int inner_solve(gkb_ctx* c, const double* f, double* x_out, double tol, int* iters) {
  Inner<T>& in = inner_of<T>(c);
  if (!in.ready) return GKB_EINVAL;
  if (c->opt.krylov == GKB_KRYLOV_FGMRES && !learned_capturing(c->learned))
    return fgmres_solve<T>(c, f, x_out, tol, iters);
  if (learned_capturing(c->learned) && c->opt.inner != GKB_INNER_JACOBI)
    return capture_solve<T>(c, f, x_out, tol, iters);
  if (c->opt.inner == GKB_INNER_LEARNED && c->learned && learned_enabled(c->learned)) {
    const int rc = learned_solve<T>(c, f, x_out, tol, iters);
    if (rc != kLearnedDeclined) return rc;
  }
  const Level<T>& L0 = in.lv[0];
  const int n = L0.g.m_full, vb = vec_blocks(n);
  hipStream_t s = c->cs;
  k_pcg_init<double, T><<<vb, kBlock, 0, s>>>(n, f, in.x, in.r, c->part[3]);
  if (c->opt.inner == GKB_INNER_JACOBI) {
    k_pcg_p0<T><<<vb, kBlock, 0, s>>>(n, in.dinv, in.r, in.z, in.p, c->part[2]);
  } else {
    vcycle<T>(c, in, 0, in.r, in.z, nullptr, nullptr);
    k_pcg_p0<T><<<vb, kBlock, 0, s>>>(n, nullptr, in.r, in.z, in.p, c->part[2]);
  }
  k_pcg_start<<<1, kFinal, 0, s>>>(in.st, c->part[3], vb, c->part[2], vb, tol, c->opt.inner_maxit);
  const int chunk = std::max(1, c->opt.check_every);
  if (c->opt.use_graphs) CK(ensure_graph<T>(c, in, chunk));
  PcgState hs;
  for (;;) {
    if (c->opt.use_graphs) {
      HIPCK(hipGraphLaunch(in.graph, s));
    } else {
      CK(pcg_iterations<T>(c, in, chunk));
    }
    HIPCK(hipMemcpyAsync(c->hbuf, in.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    std::memcpy(&hs, c->hbuf, sizeof(PcgState));
    if (hs.done) break;
  }
  k_cast<T, double><<<vb, kBlock, 0, s>>>(n, in.x, x_out);
  if (iters) *iters = hs.it;
  c->stats.inner_iterations += hs.it;
  c->stats.inner_solves += 1;
  if (hs.nonfinite) return GKB_ENAN;
  if (hs.status == -5) return GKB_EINNER;
  return GKB_OK;
}

int inner_solve_any(gkb_ctx* c, const double* f, double* x, double tol, int* iters) {
  if (c->opt.precision == GKB_MIXED) return inner_solve<float>(c, f, x, tol, iters);
  return inner_solve<double>(c, f, x, tol, iters);
}

// ---------------------------------------------------------------- GKB
//
// The run is organised around the generalized Golub-Kahan relations
// A Q = M V B, A^T V = N Q B^T, V^T M V = I, Q^T N Q = I (Section 2.1),
// N = (1/eta) I (eta > 0) or I: a bidiagonalization step produces the next
// coefficients (alpha, beta) and the M-normalised v with M v, and the
// Craig-variant update turns them into the iterates u, p through
// zeta and the direction d.  Host FP64 scalars, device vectors.

struct GkScalars {
  double ninv = 1.0;   // N^-1 = ninv I
  double alpha = 0.0;  // alpha_k
  double beta = 0.0;   // beta_k (beta_1 = ||b||_{N^-1})
  double zeta = 0.0;   // zeta_k
};

// transformation to a zero first right-hand side (Section 2):
// w0 = M^-1 (g + gamma A N^-1 r) (skipped when that is 0), b = r - A^T w0;
// returns beta_1 = ||b||_{N^-1}
int gk_transform(gkb_ctx* c, const double* gv, const double* rv, double ninv, double* beta1) {
  const Grid& G = c->g;
  const int m = G.m_full;
  hipStream_t s = c->cs;
  int its = 0;
  grad_axpy(c, rv, gv, c->eta, 1.0, c->ghat);  // ghat = g + eta A r (masked)
  k_dot<double><<<vec_blocks(m), kBlock, 0, s>>>(m, c->ghat, c->ghat, c->part[0]);
  double gg = 0.0;
  CK(host_sum(c, c->part[0], vec_blocks(m), &gg));
  if (!std::isfinite(gg)) return GKB_ENAN;
  if (gg == 0.0) k_fill<double><<<vec_blocks(m), kBlock, 0, s>>>(m, 0.0, c->w0);
  else CK(inner_solve_any(c, c->ghat, c->w0, c->opt.inner_tol, &its));
  div_axpy<double>(c, G, c->w0, rv, -1.0, 1.0, c->b, c->part[0], nullptr);
  double bb = 0.0;
  CK(host_sum(c, c->part[0], div_parts(c), &bb));
  *beta1 = std::sqrt(ninv * bb);
  return std::isfinite(*beta1) ? GKB_OK : GKB_ENAN;
}

// s = M^-1 f (inner solve), y = M s, alpha = ||s||_M by the explicit product
int gk_solve_and_norm(gkb_ctx* c, double* alpha) {
  int its = 0;
  CK(inner_solve_any(c, c->f, c->s, c->opt.inner_tol, &its));
  face_op<double, kApplyDot>(c, c->op64, c->fl0, c->s, nullptr, c->y, 0.0, c->part[0], nullptr);
  double sMs = 0.0;
  CK(host_sum(c, c->part[0], c->fl0.nparts, &sMs));
  *alpha = std::sqrt(sMs);
  return (std::isfinite(*alpha) && *alpha > 0.0) ? GKB_OK : GKB_ENAN;
}

// first column: q_1 = N^-1 b / beta_1, alpha_1 M v_1 = A q_1
int gk_first(gkb_ctx* c, GkScalars& S, double beta1) {
  const int nc = c->g.n_cells, vbc = vec_blocks(nc);
  hipStream_t s = c->cs;
  S.beta = beta1;
  k_cast<double, double><<<vbc, kBlock, 0, s>>>(nc, c->b, c->q);
  k_axpby<<<vbc, kBlock, 0, s>>>(nc, 0.0, c->q, S.ninv / beta1, c->q);
  grad_axpy(c, c->q, nullptr, 1.0, 0.0, c->f);  // f = A q_1
  return gk_solve_and_norm(c, &S.alpha);
}

// next column from A^T V = N Q B^T: beta N q_{k+1} = A^T v_k - alpha_k N q_k,
// i.e. t = N^-1 A^T v_k - alpha_k q_k, beta = ||t||_N; and from A Q = M V B:
// alpha M v_{k+1} = A q_{k+1} - beta M v_k.  *breakdown: beta at rounding
// level relative to alpha (both in the N-norm of t's two terms), the Krylov
// space is exhausted
int gk_next(gkb_ctx* c, GkScalars& S, bool* breakdown) {
  const Grid& G = c->g;
  const int nc = G.n_cells, vbc = vec_blocks(nc);
  hipStream_t s = c->cs;
  div_axpy<double>(c, G, c->v, c->q, S.ninv, -S.alpha, c->t, c->part[0], nullptr);
  double tt = 0.0;
  CK(host_sum(c, c->part[0], div_parts(c), &tt));
  const double beta = std::sqrt(tt / S.ninv);
  if (!std::isfinite(beta)) return GKB_ENAN;
  *breakdown = beta <= 1e-13 * S.alpha;
  if (*breakdown) return GKB_OK;
  S.beta = beta;
  k_cast<double, double><<<vbc, kBlock, 0, s>>>(nc, c->t, c->q);
  k_axpby<<<vbc, kBlock, 0, s>>>(nc, 0.0, c->q, 1.0 / beta, c->q);
  grad_axpy(c, c->q, c->Mv, 1.0, -beta, c->f);  // f = A q - beta M v
  return gk_solve_and_norm(c, &S.alpha);
}

// Craig-variant update with the newest column, fused with the normalisation
// of v: v = s / alpha, M v = y / alpha, zeta_k (beta_1 / alpha_1 first, then
// -(beta_k / alpha_k) zeta_{k-1}), u += zeta v; d = (q - beta d) / alpha,
// p -= zeta d
void craig_update(gkb_ctx* c, GkScalars& S, bool first, double* p) {
  const int m = c->g.m_full, nc = c->g.n_cells;
  hipStream_t s = c->cs;
  S.zeta = first ? S.beta / S.alpha : -(S.beta / S.alpha) * S.zeta;
  k_gkb_faces<<<vec_blocks(m), kBlock, 0, s>>>(m, 1.0 / S.alpha, S.zeta, c->s, c->y, c->v, c->Mv,
                                               c->u);
  k_gkb_cells<<<vec_blocks(nc), kBlock, 0, s>>>(nc, 1.0 / S.alpha, first ? 0.0 : S.beta, S.zeta,
                                                c->q, c->d, p);
}

// lower bound of the energy-norm error relative to the solution from the
// newest delay+1 zeta values (Section 2.2; the non-squared ratio), -1
// before K = delay + 1
double lower_bound_ratio(const std::vector<double>& zs, int delay, double sum_all) {
  const int K = (int)zs.size();
  if (K < delay + 1) return -1.0;
  double win = 0.0;
  for (int j = K - delay; j <= K; ++j) win += zs[j - 1] * zs[j - 1];
  return std::sqrt(win / sum_all);
}

// One GKB run for the right-hand sides (gv, rv); writes w = u_K + w0 and p.
int gkb_run(gkb_ctx* c, const double* gv, const double* rv, double tol, int delay, double* w,
            double* p, int* K_out, double* est_out) {
  const int m = c->g.m_full, nc = c->g.n_cells, vbm = vec_blocks(m), vbc = vec_blocks(nc);
  hipStream_t s = c->cs;
  GkScalars S;
  S.ninv = c->eta > 0.0 ? c->eta : 1.0;
  double beta1 = 0.0;
  CK(gk_transform(c, gv, rv, S.ninv, &beta1));
  k_fill<double><<<vbc, kBlock, 0, s>>>(nc, 0.0, p);
  k_fill<double><<<vbc, kBlock, 0, s>>>(nc, 0.0, c->d);
  k_fill<double><<<vbm, kBlock, 0, s>>>(m, 0.0, c->u);
  c->stats.history_len = 0;
  std::vector<double> zs;
  double est = 1.0, sum_all = 0.0;
  int status = GKB_MAXIT;
  if (beta1 == 0.0) {  // b = 0: w0 is the solution
    est = 0.0;
    status = GKB_OK;
  } else {
    CK(gk_first(c, S, beta1));
    for (;;) {
      craig_update(c, S, zs.empty(), p);
      zs.push_back(S.zeta);
      sum_all += S.zeta * S.zeta;
      const int K = (int)zs.size();
      const double e = lower_bound_ratio(zs, delay, sum_all);
      if (e >= 0.0) est = e;
      if (K <= 512) {
        c->stats.zeta[K - 1] = S.zeta;
        c->stats.estimate[K - 1] = e;
        c->stats.history_len = K;
      }
      if (e >= 0.0 && tol > 0.0 && e <= tol) {
        status = GKB_OK;
        break;
      }
      if (K >= c->opt.maxit) break;
      bool breakdown = false;
      CK(gk_next(c, S, &breakdown));
      if (breakdown) {
        est = 0.0;
        status = GKB_OK;
        break;
      }
    }
  }
  // w = u + w0 (non-unknown faces are zero in both)
  k_cast<double, double><<<vbm, kBlock, 0, s>>>(m, c->u, w);
  k_axpby<<<vbm, kBlock, 0, s>>>(m, 1.0, c->w0, 1.0, w);
  HIPCK(hipStreamSynchronize(s));
  if (K_out) *K_out = (int)zs.size();
  if (est_out) *est_out = est;
  c->stats.outer_iterations += (int)zs.size();
  c->stats.error_estimate = est;
  return status;
}

// FP64 saddle residual res = [g - W w - A p; r - A^T w] and its norms.  On
// an assembled system with central scaling the iteration works in the
// scaled space; user_space = true takes the user's unscaled operators (the
// public gkb_residual), false the iteration's.
int residual_impl(gkb_ctx* c, const double* gv, const double* rv, const double* w, const double* p,
                  double* res_w, double* res_r, double* norms, bool user_space = false) {
  const Grid& G = c->g;
  hipStream_t s = c->cs;
  int nw = 0, nr = 0;
  if (c->csr) {
    CsrOps<double> o = c->csr64;
    if (user_space) o.sw = o.sp = nullptr;
    nw = vec_blocks(o.m);
    nr = vec_blocks(o.n);
    k_csr_resid_w<<<nw, kBlock, 0, s>>>(o, gv, w, p, res_w, c->part[0], c->part[1]);
    k_csr_div<double><<<nr, kBlock, 0, s>>>(o, w, rv, -1.0, 1.0, res_r ? res_r : c->t, c->part[2],
                                            c->part[3]);
  } else {
    Op<double> opW = c->op64;
    opW.eta = 0.0;
    const FaceLaunch& fl = c->fl0;
    const bool vm = opW.mu != nullptr;
    if (G.dim == 2) {
      if (vm) k_resid_w<2, true><<<fl.grid, kBlock, 0, s>>>(opW, gv, w, p, res_w, fl.kz, fl.zchunks, c->part[0], c->part[1]);
      else k_resid_w<2, false><<<fl.grid, kBlock, 0, s>>>(opW, gv, w, p, res_w, fl.kz, fl.zchunks, c->part[0], c->part[1]);
    } else {
      if (vm) k_resid_w<3, true><<<fl.grid, kBlock, 0, s>>>(opW, gv, w, p, res_w, fl.kz, fl.zchunks, c->part[0], c->part[1]);
      else k_resid_w<3, false><<<fl.grid, kBlock, 0, s>>>(opW, gv, w, p, res_w, fl.kz, fl.zchunks, c->part[0], c->part[1]);
    }
    div_axpy<double>(c, G, w, rv, -1.0, 1.0, res_r ? res_r : c->t, c->part[2], c->part[3]);
    nw = fl.gparts;
    nr = cell_parts(G);
  }
  double rw = 0, ggw = 0, rrr = 0, rr2 = 0;
  CK(host_sum(c, c->part[0], nw, &rw));
  CK(host_sum(c, c->part[1], nw, &ggw));
  CK(host_sum(c, c->part[2], nr, &rrr));
  CK(host_sum(c, c->part[3], nr, &rr2));
  norms[0] = std::sqrt(rw + rrr);
  norms[1] = std::sqrt(rw);
  norms[2] = std::sqrt(rrr);
  norms[3] = std::sqrt(ggw + rr2);
  return GKB_OK;
}

// GKB as a preconditioner (Section 3 offers GKB as a solver or as a
// preconditioner): restarted flexible GMRES on the whole saddle system
// K [w; p] = [g; r], right preconditioned by one GKB run per step (the
// lower-bound tolerance tol, delay and maxit of the options), modified
// Gram-Schmidt and Givens rotations on the host in FP64, every vector
// operation on the device.  Stops when the least-squares residual estimate,
// or the true FP64 residual at a restart, is <= refine_tol ||[g; r]||, or
// after max_sweeps steps (GKB_MAXIT).
int precond_solve(gkb_ctx* c, const double* gv, const double* rv, double tol, int delay,
                  double* w, double* p, int* K_out, double* est_out) {
  const int m = c->g.m_full, nc = c->g.n_cells;
  const long N = (long)m + nc;
  const int R = c->opt.outer_restart, maxit = c->opt.max_sweeps;
  const double rtol = c->opt.refine_tol;
  hipStream_t s = c->cs;
  const int vbN = vec_blocks((int)N), vbm = vec_blocks(m), vbc = vec_blocks(nc);
  auto V = [&](int j) { return c->ov + (size_t)j * N; };
  auto Z = [&](int j) { return c->oz + (size_t)j * N; };
  auto pdot = [&](const double* a, const double* b, double* out) {
    k_dot<double><<<vbN, kBlock, 0, s>>>((int)N, a, b, c->part[4]);
    return host_sum(c, c->part[4], vbN, out);
  };
  std::vector<double> H((size_t)(R + 1) * R, 0.0), cs(R), sn(R), gr(R + 1), y(R);
  k_fill<double><<<vbm, kBlock, 0, s>>>(m, 0.0, w);
  k_fill<double><<<vbc, kBlock, 0, s>>>(nc, 0.0, p);
  int it = 0, status = GKB_MAXIT, K = 0;
  double est = 0.0, norms[4];
  for (;;) {
    // true residual r = b - K x into V_0
    CK(residual_impl(c, gv, rv, w, p, V(0), V(0) + m, norms));
    const double beta = norms[0], bnorm = norms[3];
    c->stats.residual = bnorm > 0.0 ? beta / bnorm : 0.0;
    if (!std::isfinite(beta)) return GKB_ENAN;
    if (beta <= rtol * bnorm) {
      status = GKB_OK;
      break;
    }
    if (it >= maxit) break;
    k_axpby<<<vbN, kBlock, 0, s>>>((int)N, 0.0, V(0), 1.0 / beta, V(0));
    std::fill(gr.begin(), gr.end(), 0.0);
    gr[0] = beta;
    int k = 0;
    bool conv = false;
    for (int j = 0; j < R && it < maxit; ++j) {
      // z_j = GKB(v_j): one run on the right-hand side (faces, cells) of v_j
      const int rc = gkb_run(c, V(j), V(j) + m, tol, delay, Z(j), Z(j) + m, &K, &est);
      c->stats.sweeps += 1;
      if (rc < 0) return rc;
      // w = K z_j, formed as -(0 - K z_j) by the residual kernels
      CK(residual_impl(c, c->ozero, c->ozero + m, Z(j), Z(j) + m, V(j + 1), V(j + 1) + m,
                       norms));
      double* wv = V(j + 1);
      k_axpby<<<vbN, kBlock, 0, s>>>((int)N, 0.0, wv, -1.0, wv);
      for (int i = 0; i <= j; ++i) {
        double hij = 0.0;
        CK(pdot(wv, V(i), &hij));
        H[(size_t)i * R + j] = hij;
        k_axpby<<<vbN, kBlock, 0, s>>>((int)N, -hij, V(i), 1.0, wv);
      }
      double ww = 0.0;
      CK(pdot(wv, wv, &ww));
      const double hn = std::sqrt(ww);
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * R + j], b = H[(size_t)(i + 1) * R + j];
        H[(size_t)i * R + j] = cs[i] * a + sn[i] * b;
        H[(size_t)(i + 1) * R + j] = -sn[i] * a + cs[i] * b;
      }
      const double a = H[(size_t)j * R + j], rr = std::sqrt(a * a + hn * hn);
      ++it;
      if (!std::isfinite(rr)) return GKB_ENAN;
      if (rr == 0.0) break;  // K z_j adds nothing: restart
      cs[j] = a / rr;
      sn[j] = hn / rr;
      H[(size_t)j * R + j] = rr;
      gr[j + 1] = -sn[j] * gr[j];
      gr[j] = cs[j] * gr[j];
      k = j + 1;
      if (std::fabs(gr[j + 1]) <= rtol * bnorm || hn == 0.0) {
        conv = true;
        break;
      }
      k_axpby<<<vbN, kBlock, 0, s>>>((int)N, 0.0, wv, 1.0 / hn, wv);
    }
    for (int i = k - 1; i >= 0; --i) {
      double v = gr[i];
      for (int l = i + 1; l < k; ++l) v -= H[(size_t)i * R + l] * y[l];
      y[i] = v / H[(size_t)i * R + i];
    }
    for (int l = 0; l < k; ++l) {
      k_axpby<<<vbm, kBlock, 0, s>>>(m, y[l], Z(l), 1.0, w);
      k_axpby<<<vbc, kBlock, 0, s>>>(nc, y[l], Z(l) + m, 1.0, p);
    }
    if (conv) {
      CK(residual_impl(c, gv, rv, w, p, V(0), V(0) + m, norms));
      c->stats.residual = norms[3] > 0.0 ? norms[0] / norms[3] : 0.0;
      status = GKB_OK;
      break;
    }
  }
  HIPCK(hipStreamSynchronize(s));
  c->stats.outer_krylov_iterations = it;
  if (K_out) *K_out = K;
  if (est_out) *est_out = est;
  return status;
}

// ------------------------------------------------------------- setup

void edge_viscosity(const Grid& g, const std::vector<double>& mu, int B, std::vector<double>& out) {
  int ex[3];
  for (int a = 0; a < 3; ++a) ex[a] = g.n[a] + (a != B ? 1 : 0);
  if (g.dim == 2) ex[2] = 1;
  out.assign((size_t)ex[0] * ex[1] * ex[2], 0.0);
  for (int k = 0; k < ex[2]; ++k)
    for (int j = 0; j < ex[1]; ++j)
      for (int i = 0; i < ex[0]; ++i) {
        const int E[3] = {i, j, k};
        double sum = 0.0;
        int cnt = 0;
        // cells touching the edge: along axes != B the two cells E-1, E
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          if (a == B || (g.dim == 2 && a == 2)) {
            lo[a] = hi[a] = E[a];
          } else {
            lo[a] = E[a] - 1;
            hi[a] = E[a];
          }
        }
        for (int kk = lo[2]; kk <= hi[2]; ++kk)
          for (int jj = lo[1]; jj <= hi[1]; ++jj)
            for (int ii = lo[0]; ii <= hi[0]; ++ii) {
              if (ii < 0 || jj < 0 || kk < 0 || ii >= g.n[0] || jj >= g.n[1] || kk >= g.n[2])
                continue;
              sum += mu[((size_t)kk * g.n[1] + jj) * g.n[0] + ii];
              ++cnt;
            }
        out[((size_t)k * ex[1] + j) * ex[0] + i] = cnt ? sum / cnt : 1.0;
      }
}

// Host <-> device copy ordered on the context's stream and complete on return.
// The context stream is non-blocking, so it is not ordered with the null
// stream that a plain hipMemcpy uses (a pageable upload may also return
// before its DMA has landed).
int copy_sync(gkb_ctx* c, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  HIPCK(hipMemcpyAsync(dst, src, bytes, kind, c->cs));
  HIPCK(hipStreamSynchronize(c->cs));
  return GKB_OK;
}

template <typename T>
int upload(gkb_ctx* c, const std::vector<double>& h, T** out) {
  std::vector<T> tmp(h.begin(), h.end());
  CK(c->mem.arr(out, tmp.size()));
  CK(copy_sync(c, *out, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
  return GKB_OK;
}

template <typename T>
Op<T> make_op(const Grid& g, double eta, const Coef<T>& cf, bool varmu) {
  Op<T> op;
  op.g = g;
  op.eta = T(eta);
  op.ih2 = T(1.0 / (g.h * g.h));
  op.ih = T(1.0 / g.h);
  op.mu = varmu ? cf.mu : nullptr;
  for (int b = 0; b < 3; ++b) op.mue[b] = varmu ? cf.mue[b] : nullptr;
  return op;
}

// Cholesky-based inverse of an SPD matrix (row-major, in place); false if
// not positive definite
bool spd_inverse(std::vector<double>& A, int n) {
  // Cholesky A = L L^T (row-major L; inner products over contiguous rows)
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    const double* Lj = &L[(size_t)j * n];
    double dsum = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) dsum -= Lj[k] * Lj[k];
    if (!(dsum > 0.0)) return false;
    const double ljj = std::sqrt(dsum);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      const double* Li = &L[(size_t)i * n];
      double sum = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) sum -= Li[k] * Lj[k];
      L[(size_t)i * n + j] = sum / ljj;
    }
  }
  // X = L^-1, row by row: row i of L X = e_i gives
  // X_i = (e_i - sum_{l < i} L[i][l] X_l) / L[i][i], with rows X_l nonzero
  // in columns 0..l only (contiguous row updates)
  std::vector<double> X((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    const double* Li = &L[(size_t)i * n];
    double* Xi = &X[(size_t)i * n];
    for (int l = 0; l < i; ++l) {
      const double a = Li[l];
      const double* Xl = &X[(size_t)l * n];
      for (int k = 0; k <= l; ++k) Xi[k] -= a * Xl[k];
    }
    Xi[i] = 1.0;
    const double inv = 1.0 / Li[i];
    for (int k = 0; k <= i; ++k) Xi[k] *= inv;
  }
  // A^-1 = X^T X as a sum of outer products of the rows of X (lower part,
  // then mirrored)
  for (size_t e = 0; e < (size_t)n * n; ++e) A[e] = 0.0;
  for (int k = 0; k < n; ++k) {
    const double* Xk = &X[(size_t)k * n];
    for (int i = 0; i <= k; ++i) {
      const double a = Xk[i];
      double* Ai = &A[(size_t)i * n];
      for (int j = 0; j <= i; ++j) Ai[j] += a * Xk[j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) A[(size_t)j * n + i] = A[(size_t)i * n + j];
  return true;
}

// Hybrid smoother set-up on every level but the coarsest (FP64):
// diag(C^T W C) by probing (27 (3D) or 9 (2D) edge classes per component,
// see k_edge_probe), its inverse, and the edge-sweep weight
// omega_e = 1.5 / (1.05 lambda) from 30 power steps on D_e^-1 C^T W C
// (lambda underestimates the top eigenvalue slightly, hence 1.05; 1.5 / lambda
// was the fastest of 0.7, 1.0, 1.5, 1.8 on the 128^3 lid-driven problem).
template <int DIM>
int edge_setup_level(gkb_ctx* c, int l, double* psi, double* t, double* dg, double* cf,
                     double* y) {
  const Grid& g = c->grids[l];
  hipStream_t s = c->cs;
  const Op<double> opW = make_op<double>(g, 0.0, c->coef64[l], c->varmu);
  const FaceLaunch fl = face_launch(g, 4, c->opt.stencil);
  const long ne = (long)edge_comps<DIM>() * g.n_cells;
  const int m = g.m_full;
  const dim3 cg = cell_grid(g);
  const int eb = (int)std::min<long>(4096, (ne + kBlock - 1) / kBlock);
  k_fill<double><<<vec_blocks((int)ne), kBlock, 0, s>>>((int)ne, 0.0, dg);
  for (int a = 0; a < edge_comps<DIM>(); ++a)
    for (int cz = 0; cz < (DIM == 3 ? 3 : 1); ++cz)
      for (int cy = 0; cy < 3; ++cy)
        for (int cx = 0; cx < 3; ++cx) {
          k_edge_probe<DIM><<<cg, kBlock, 0, s>>>(g, a, cx, cy, cz, psi);
          k_fill<double><<<vec_blocks(m), kBlock, 0, s>>>(m, 0.0, cf);
          k_curl_add<double, DIM><<<cg, kBlock, 0, s>>>(g, psi, cf, nullptr);
          face_op<double, kApply>(c, opW, fl, cf, nullptr, y, 0.0, nullptr, nullptr);
          k_edge_ct<double, DIM><<<cg, kBlock, 0, s>>>(g, y, nullptr, 1.0, t, nullptr);
          k_edge_collect<<<eb, kBlock, 0, s>>>(ne, psi, t, dg);
        }
  std::vector<double> dh(ne);
  HIPCK(hipMemcpyAsync(dh.data(), dg, ne * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  for (auto& v : dh) v = v > 0.0 ? 1.0 / v : 0.0;
  CK(copy_sync(c, dg, dh.data(), ne * sizeof(double), hipMemcpyHostToDevice));
  // power iteration from D_e^-1 C^T (seeded random faces)
  std::vector<double> f0(m);
  unsigned sd = 54321u;
  for (auto& v : f0) {
    sd = sd * 1664525u + 1013904223u;
    v = (sd >> 8) * (1.0 / 16777216.0) - 0.5;
  }
  CK(copy_sync(c, cf, f0.data(), m * sizeof(double), hipMemcpyHostToDevice));
  k_edge_ct<double, DIM><<<cg, kBlock, 0, s>>>(g, cf, dg, 1.0, psi, nullptr);
  double lam = 1.0;
  for (int it = 0; it < 30; ++it) {
    k_fill<double><<<vec_blocks(m), kBlock, 0, s>>>(m, 0.0, cf);
    k_curl_add<double, DIM><<<cg, kBlock, 0, s>>>(g, psi, cf, nullptr);
    face_op<double, kApply>(c, opW, fl, cf, nullptr, y, 0.0, nullptr, nullptr);
    k_edge_ct<double, DIM><<<cg, kBlock, 0, s>>>(g, y, dg, 1.0, t, nullptr);
    double tt = 0.0, xx = 0.0;
    k_dot<double><<<vec_blocks((int)ne), kBlock, 0, s>>>((int)ne, t, t, c->part[0]);
    CK(host_sum(c, c->part[0], vec_blocks((int)ne), &tt));
    k_dot<double><<<vec_blocks((int)ne), kBlock, 0, s>>>((int)ne, psi, psi, c->part[1]);
    CK(host_sum(c, c->part[1], vec_blocks((int)ne), &xx));
    if (!(tt > 0.0) || !(xx > 0.0)) break;
    lam = std::sqrt(tt / xx);
    k_axpby<<<vec_blocks((int)ne), kBlock, 0, s>>>((int)ne, 1.0 / std::sqrt(tt), t, 0.0, psi);
  }
  c->omega_e[l] = 1.5 / (1.05 * lam);
  c->edinv_h[l] = std::move(dh);
  return GKB_OK;
}

int edge_setup(gkb_ctx* c) {
  const int L = c->L;
  c->omega_e.assign(L, 0.0);
  c->edinv_h.assign(L, std::vector<double>());
  if (L < 2) return GKB_OK;
  const Grid& g0 = c->grids[0];
  const long ne = (long)(g0.dim == 3 ? 3 : 1) * g0.n_cells;
  double *psi, *t, *dg, *cf, *y;
  CK(c->mem.arr(&psi, ne));
  CK(c->mem.arr(&t, ne));
  CK(c->mem.arr(&dg, ne));
  CK(c->mem.arr(&cf, g0.m_full));
  CK(c->mem.arr(&y, g0.m_full));
  for (int l = 0; l < L - 1; ++l) {
    if (g0.dim == 2) CK(edge_setup_level<2>(c, l, psi, t, dg, cf, y));
    else CK(edge_setup_level<3>(c, l, psi, t, dg, cf, y));
  }
  return GKB_OK;
}

template <typename T>
int build_inner(gkb_ctx* c, Inner<T>& in, const std::vector<Coef<T>>& coef) {
  const int L = c->L;
  in.lv.resize(L);
  for (int l = 0; l < L; ++l) {
    Level<T>& lv = in.lv[l];
    lv.g = c->grids[l];
    lv.op = make_op<T>(lv.g, c->eta, coef[l], c->varmu);
    lv.omega = c->omega[l];
    if (c->csr) {
      lv.fl = FaceLaunch{};
      lv.fl.nparts = lv.fl.gparts = vec_blocks(lv.g.m_full);
    } else {
      lv.fl = face_launch(lv.g, 4, c->opt.stencil);
    }
    const int m = lv.g.m_full;
    if (l > 0) {
      CK(c->mem.arr(&lv.b, m));
      CK(c->mem.arr(&lv.x, m));
    }
    CK(c->mem.arr(&lv.t, m));
    CK(c->mem.arr(&lv.rb, m));
    if (l >= 1 && l < L - 1) {
      CK(c->mem.arr(&lv.dinv, m));
      face_op<T, kDiag>(c, lv.op, lv.fl, nullptr, nullptr, lv.dinv, T(0), nullptr, nullptr);
      std::vector<T> dh(m);
      CK(copy_sync(c, dh.data(), lv.dinv, m * sizeof(T), hipMemcpyDeviceToHost));
      for (auto& v : dh) v = v != T(0) ? T(1) / v : T(0);
      CK(copy_sync(c, lv.dinv, dh.data(), m * sizeof(T), hipMemcpyHostToDevice));
    }
    if (l < L - 1 && l < (int)c->edinv_h.size() && !c->edinv_h[l].empty()) {
      const std::vector<double>& dh = c->edinv_h[l];
      CK(upload<T>(c, dh, &lv.edinv));
      lv.omega_e = c->omega_e[l];
    }
  }
  const int m = c->g.m_full;
  CK(c->mem.arr(&in.x, m));
  CK(c->mem.arr(&in.r, m));
  CK(c->mem.arr(&in.z, m));
  CK(c->mem.arr(&in.p, m));
  if (sizeof(T) == 4 && c->fl0.tiled && c->opt.inner != GKB_INNER_JACOBI) CK(c->mem.arr(&in.p2, m));
  CK(c->mem.arr(&in.q, m));
  CK(c->mem.arr(&in.rprev, m));
  CK(c->mem.arr(&in.st, 1));
  if (c->opt.krylov == GKB_KRYLOV_FGMRES) {
    const int R = c->opt.fgmres_restart;
    CK(c->mem.arr(&in.gm_V, (size_t)(R + 1) * m));
    CK(c->mem.arr(&in.gm_Z, (size_t)R * m));
    CK(c->mem.arr(&in.gm_fs, 1));
    CK(c->mem.arr(&in.gm_cyc, 1));
    CK(c->mem.arr(&in.gm_part, (size_t)(R + 1) * vec_blocks(m)));
  }
  // Jacobi preconditioner 1/diag(M) (0 at non-unknown faces)
  CK(c->mem.arr(&in.dinv, m));
  face_op<T, kDiag>(c, in.lv[0].op, in.lv[0].fl, nullptr, nullptr, in.dinv, T(0), nullptr, nullptr);
  std::vector<T> dh(m);
  HIPCK(hipMemcpyAsync(dh.data(), in.dinv, m * sizeof(T), hipMemcpyDeviceToHost, c->cs));
  HIPCK(hipStreamSynchronize(c->cs));
  for (auto& v : dh) v = v != T(0) ? T(1) / v : T(0);
  CK(copy_sync(c, in.dinv, dh.data(), m * sizeof(T), hipMemcpyHostToDevice));
  in.ready = true;
  return GKB_OK;
}

int setup_impl(gkb_ctx* c, const gkb_grid* grid, const double* visc, double eta,
               const gkb_options* opt) {
  c->opt = *opt;
  c->eta = eta;
  c->mem.cap = opt->max_workspace_bytes;
  c->us = static_cast<hipStream_t>(opt->hip_stream);
  HIPCK(hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking));
  c->mem.s = c->cs;
  HIPCK(hipEventCreateWithFlags(&c->ev, hipEventDisableTiming));
  int n[3] = {grid->n[0], grid->n[1], grid->dim == 3 ? grid->n[2] : 1};
  c->g = make_grid(grid->dim, n, grid->h, grid->bc, grid->pin_cell);
  c->varmu = visc != nullptr;
  {
    // AUTO transfers: SMOOTH while the grad-div term is weak against the
    // viscous one, eta <= 100 mu_ref (mu_ref: geometric mean viscosity)
    double mu_ref = 1.0;
    if (visc) {
      double sl = 0.0;
      for (int i = 0; i < c->g.n_cells; ++i) sl += std::log(visc[i]);
      mu_ref = std::exp(sl / c->g.n_cells);
    }
    c->smooth_transfer = opt->mg_transfer == GKB_TRANSFER_SMOOTH ||
                         (opt->mg_transfer == GKB_TRANSFER_AUTO && eta <= 100.0 * mu_ref);
  }
  // levels
  int L = opt->mg_levels;
  if (opt->inner == GKB_INNER_JACOBI) L = 1;
  if (L <= 0) {
    L = 1;
    int nn[3] = {n[0], n[1], n[2]};
    // coarsen while the current level has more than 2000 faces and every
    // axis halves to at least 2 cells (the coarsest level is solved densely)
    for (;;) {
      bool ok = true;
      long mf = 0;
      for (int cc = 0; cc < grid->dim; ++cc) {
        long e = 1;
        for (int a = 0; a < grid->dim; ++a) e *= nn[a] + (a == cc ? 1 : 0);
        mf += e;
      }
      for (int a = 0; a < grid->dim; ++a) ok = ok && (nn[a] % 2 == 0) && (nn[a] >= 4);
      if (!ok || mf <= 2000 || L >= kMaxLevels) break;
      for (int a = 0; a < grid->dim; ++a) nn[a] /= 2;
      ++L;
    }
  }
  for (int l = 1; l < L; ++l)
    for (int a = 0; a < grid->dim; ++a)
      if ((n[a] >> (l - 1)) % 2 != 0 || (n[a] >> l) < 2) return GKB_EINVAL;
  c->L = L;
  std::vector<std::vector<double>> mus(L);
  for (int l = 0; l < L; ++l) {
    int nl[3] = {n[0] >> l, n[1] >> l, grid->dim == 3 ? (n[2] >> l) : 1};
    int pin = -1;
    if (grid->pin_cell >= 0) {
      const int pi = grid->pin_cell % n[0], pj = (grid->pin_cell / n[0]) % n[1],
                pk = grid->pin_cell / (n[0] * n[1]);
      pin = ((pk >> l) * nl[1] + (pj >> l)) * nl[0] + (pi >> l);
      if (grid->dim == 2) pin = (pj >> l) * nl[0] + (pi >> l);
    }
    c->grids.push_back(make_grid(grid->dim, nl, grid->h * (double)(1 << l), grid->bc, pin));
    const Grid& g = c->grids.back();
    mus[l].assign(g.n_cells, 1.0);
    if (c->varmu) {
      if (l == 0) {
        std::memcpy(mus[0].data(), visc, sizeof(double) * g.n_cells);
      } else {
        const Grid& f = c->grids[l - 1];
        const int dz = grid->dim == 3 ? 2 : 1;
        for (int k = 0; k < g.n[2]; ++k)
          for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
              double s = 0;
              for (int kk = 0; kk < dz; ++kk)
                for (int jj = 0; jj < 2; ++jj)
                  for (int ii = 0; ii < 2; ++ii)
                    s += mus[l - 1][((size_t)(dz * k + kk) * f.n[1] + 2 * j + jj) * f.n[0] + 2 * i + ii];
              mus[l][((size_t)k * g.n[1] + j) * g.n[0] + i] = s / (dz * 4);
            }
      }
    }
  }
  c->coef64.resize(L);
  c->coef32.resize(L);
  if (c->varmu) {
    for (int l = 0; l < L; ++l) {
      const Grid& g = c->grids[l];
      CK(upload<double>(c, mus[l], &c->coef64[l].mu));
      CK(upload<float>(c, mus[l], &c->coef32[l].mu));
      for (int b = 0; b < 3; ++b) {
        if (g.dim == 2 && b != 2) continue;
        std::vector<double> e;
        edge_viscosity(g, mus[l], b, e);
        CK(upload<double>(c, e, &c->coef64[l].mue[b]));
        CK(upload<float>(c, e, &c->coef32[l].mue[b]));
      }
    }
  }
  c->op64 = make_op<double>(c->g, eta, c->coef64[0], c->varmu);
  c->op32 = make_op<float>(c->g, eta, c->coef32[0], c->varmu);
  c->fl0 = face_launch(c->g, 4, c->opt.stencil);
  // partial buffers: the largest reduction launch over all levels
  int maxp = 0;
  for (int l = 0; l < L; ++l) {
    maxp = std::max(maxp, face_launch(c->grids[l], 4, c->opt.stencil).nparts);
    maxp = std::max(maxp, face_launch(c->grids[l], 4, 1).nparts);
    const dim3 tg = transfer_grid(c->grids[l]);  // learned unpack partials
    maxp = std::max(maxp, (int)(tg.x * tg.z));
    maxp = std::max(maxp, cell_parts(c->grids[l]));
    maxp = std::max(maxp, vec_blocks(c->grids[l].m_full));
  }
  c->maxparts = maxp;
  for (int i = 0; i < kSlots; ++i) CK(c->mem.arr(&c->part[i], maxp));
  CK(c->mem.arr(&c->dscal, 8));
  HIPCK(hipHostMalloc(reinterpret_cast<void**>(&c->hbuf), 4096, hipHostMallocDefault));
  const int m = c->g.m_full, nc = c->g.n_cells;
  double** fv[] = {&c->ghat, &c->w0, &c->u, &c->v, &c->Mv, &c->s, &c->y, &c->f, &c->rw, &c->dw};
  for (auto pp : fv) CK(c->mem.arr(pp, m));
  double** cv[] = {&c->b, &c->q, &c->d, &c->t, &c->rr, &c->dp};
  for (auto pp : cv) CK(c->mem.arr(pp, nc));
  if (opt->refine_tol > 0.0) {
    CK(c->mem.arr(&c->wbest, m));
    CK(c->mem.arr(&c->pbest, nc));
  }
  if (opt->method == GKB_METHOD_PRECOND) {
    const size_t pair = (size_t)m + nc, R = (size_t)opt->outer_restart;
    CK(c->mem.arr(&c->ov, (R + 1) * pair));
    CK(c->mem.arr(&c->oz, R * pair));
    CK(c->mem.arr(&c->ozero, pair));
  }
  // Jacobi weights by power iteration on D^-1 M_l (FP64), omega = 1.6 / (1.05 lambda)
  c->omega.assign(L, 0.8);
  for (int l = 0; l < L - (L > 1 ? 1 : 0); ++l) {
    const Grid& g = c->grids[l];
    Op<double> op = make_op<double>(g, eta, c->coef64[l], c->varmu);
    FaceLaunch fl = face_launch(g, 4, c->opt.stencil);
    double *xa, *ya;
    CK(c->mem.arr(&xa, g.m_full));
    CK(c->mem.arr(&ya, g.m_full));
    std::vector<double> x0(g.m_full);
    unsigned s = 12345u;
    for (auto& v : x0) {
      s = s * 1664525u + 1013904223u;
      v = 0.5 + (s >> 8) * (1.0 / 16777216.0);
    }
    CK(copy_sync(c, xa, x0.data(), g.m_full * sizeof(double), hipMemcpyHostToDevice));
    double lam = 1.0;
    for (int it = 0; it < 40; ++it) {
      face_op<double, kDinvM>(c, op, fl, xa, nullptr, ya, 0.0, c->part[0], nullptr);
      double yy = 0.0;
      k_dot<double><<<vec_blocks(g.m_full), kBlock, 0, c->cs>>>(g.m_full, xa, xa, c->part[1]);
      double xx = 0.0;
      CK(host_sum(c, c->part[0], fl.nparts, &yy));
      CK(host_sum(c, c->part[1], vec_blocks(g.m_full), &xx));
      lam = std::sqrt(yy / xx);
      k_axpby<<<vec_blocks(g.m_full), kBlock, 0, c->cs>>>(g.m_full, 1.0 / std::sqrt(yy), ya, 0.0, xa);
    }
    c->omega[l] = 1.6 / (1.05 * lam);
  }
  if (opt->smoother == GKB_SMOOTH_HYBRID && opt->inner != GKB_INNER_JACOBI) CK(edge_setup(c));
  // coarsest level: dense FP64 inverse of M on the unknown faces
  if (opt->inner != GKB_INNER_JACOBI) {
    const Grid& g = c->grids[L - 1];
    const int mcf = g.m_full;
    if (mcf > 4096) return GKB_EINVAL;  // coarsest grid too large for a dense solve
    Op<double> op = make_op<double>(g, eta, c->coef64[L - 1], c->varmu);
    FaceLaunch fl = face_launch(g, 4);
    double *e, *col, *dg;
    CK(c->mem.arr(&e, mcf));
    CK(c->mem.arr(&col, mcf));
    CK(c->mem.arr(&dg, mcf));
    face_op<double, kDiag>(c, op, fl, nullptr, nullptr, dg, 0.0, nullptr, nullptr);
    std::vector<double> dgh(mcf);
    HIPCK(hipMemcpyAsync(dgh.data(), dg, mcf * sizeof(double), hipMemcpyDeviceToHost, c->cs));
    HIPCK(hipStreamSynchronize(c->cs));
    std::vector<int> idx;
    for (int i = 0; i < mcf; ++i)
      if (dgh[i] != 0.0) idx.push_back(i);
    const int nu = (int)idx.size();
    std::vector<double> Mfull((size_t)mcf * mcf);
    std::vector<double> one(1, 1.0);
    for (int jj = 0; jj < mcf; ++jj) {
      if (dgh[jj] == 0.0) continue;
      k_fill<double><<<vec_blocks(mcf), kBlock, 0, c->cs>>>(mcf, 0.0, e);
      HIPCK(hipMemcpyAsync(e + jj, one.data(), sizeof(double), hipMemcpyHostToDevice, c->cs));
      face_op<double, kApply>(c, op, fl, e, nullptr, col, 0.0, nullptr, nullptr);
      HIPCK(hipMemcpyAsync(&Mfull[(size_t)jj * mcf], col, mcf * sizeof(double),
                           hipMemcpyDeviceToHost, c->cs));
    }
    HIPCK(hipStreamSynchronize(c->cs));
    std::vector<double> Mu((size_t)nu * nu);
    for (int a = 0; a < nu; ++a)
      for (int b2 = 0; b2 < nu; ++b2) Mu[(size_t)a * nu + b2] = Mfull[(size_t)idx[b2] * mcf + idx[a]];
    if (!spd_inverse(Mu, nu)) return GKB_EINVAL;
    std::vector<double> Minv((size_t)mcf * mcf, 0.0);
    for (int a = 0; a < nu; ++a)
      for (int b2 = 0; b2 < nu; ++b2) Minv[(size_t)idx[a] * mcf + idx[b2]] = Mu[(size_t)a * nu + b2];
    CK(c->mem.arr(&c->Minv, (size_t)mcf * mcf));
    CK(copy_sync(c, c->Minv, Minv.data(), Minv.size() * sizeof(double), hipMemcpyHostToDevice));
    c->mc = mcf;
  }
  if (opt->precision == GKB_MIXED) CK(build_inner<float>(c, c->in32, c->coef32));
  else CK(build_inner<double>(c, c->in64, c->coef64));
  if (opt->inner != GKB_INNER_JACOBI) CK(learned_create(c));
  if (opt->cnn_weights) {
    if (gkb_cnn_load(opt->cnn_weights, &c->owned_net) != GKB_OK) return GKB_EINVAL;
    CK(gkb_attach_cnn(c, c->owned_net));
  }
  c->opt.cnn_weights = nullptr;  // the path is not kept
  HIPCK(hipStreamSynchronize(c->cs));
  c->stats = gkb_stats_t{};
  return GKB_OK;
}

// ----------------------------------------------------- assembled systems

// checks of a host CSR matrix with `rows` rows and column indices below
// `cols`: monotone row pointers starting at 0, columns in range, finite values
bool csr_valid(int rows, int cols, const int* ptr, const int* col, const double* val) {
  if (rows < 1 || cols < 1 || !ptr || !col || !val || ptr[0] != 0) return false;
  for (int i = 0; i < rows; ++i)
    if (ptr[i + 1] < ptr[i]) return false;
  const long nnz = ptr[rows];
  for (long e = 0; e < nnz; ++e)
    if (col[e] < 0 || col[e] >= cols || !std::isfinite(val[e])) return false;
  return true;
}

template <typename T>
int upload_csr(gkb_ctx* c, int rows, const std::vector<int>& ptr, const std::vector<int>& col,
               const std::vector<double>& val, CsrMat<T>* out) {
  int *dp = nullptr, *dc = nullptr;
  T* dv = nullptr;
  CK(c->mem.arr(&dp, ptr.size()));
  CK(c->mem.arr(&dc, std::max<size_t>(col.size(), 1)));
  CK(copy_sync(c, dp, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice));
  if (!col.empty()) CK(copy_sync(c, dc, col.data(), col.size() * sizeof(int), hipMemcpyHostToDevice));
  CK(upload<T>(c, val.empty() ? std::vector<double>(1, 0.0) : val, &dv));
  out->rows = rows;
  out->ptr = dp;
  out->col = dc;
  out->val = dv;
  return GKB_OK;
}

int setup_csr_impl(gkb_ctx* c, const gkb_csr* sys, double eta, int scaling, const gkb_options* opt) {
  c->opt = *opt;
  c->eta = eta;
  c->csr = true;
  c->mem.cap = opt->max_workspace_bytes;
  c->us = static_cast<hipStream_t>(opt->hip_stream);
  HIPCK(hipStreamCreateWithFlags(&c->cs, hipStreamNonBlocking));
  c->mem.s = c->cs;
  HIPCK(hipEventCreateWithFlags(&c->ev, hipEventDisableTiming));
  const int m = sys->m, n = sys->n;
  // the vector kernels see an m-long velocity and an n-long pressure array
  Grid G{};
  G.dim = 0;
  G.pin = -1;
  G.m_full = m;
  G.n_cells = n;
  G.h = 1.0;
  c->g = G;
  c->grids.assign(1, G);
  c->L = 1;
  c->coef64.resize(1);
  c->coef32.resize(1);
  c->omega.assign(1, 0.8);
  // host copies: W, A and the transpose of A (counting sort by column)
  const long nw = sys->w_rowptr[m], na = sys->a_rowptr[m];
  std::vector<int> wp(sys->w_rowptr, sys->w_rowptr + m + 1), wc(sys->w_col, sys->w_col + nw);
  std::vector<double> wv(sys->w_val, sys->w_val + nw);
  std::vector<int> ap(sys->a_rowptr, sys->a_rowptr + m + 1), ac(sys->a_col, sys->a_col + na);
  std::vector<double> av(sys->a_val, sys->a_val + na);
  std::vector<int> tp(n + 1, 0), tc(na);
  std::vector<double> tv(na);
  for (long e = 0; e < na; ++e) tp[ac[e] + 1] += 1;
  for (int k = 0; k < n; ++k) tp[k + 1] += tp[k];
  {
    std::vector<int> fill(tp.begin(), tp.end() - 1);
    for (int i = 0; i < m; ++i)
      for (int e = ap[i]; e < ap[i + 1]; ++e) {
        const int k = ac[e];
        tc[fill[k]] = i;
        tv[fill[k]] = av[e];
        fill[k] += 1;
      }
  }
  // diag(W) > 0 (Jacobi, scaling) and, with scaling, R = diag(A^T D^-1 A) > 0
  std::vector<double> dw(m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int e = wp[i]; e < wp[i + 1]; ++e)
      if (wc[e] == i) dw[i] += wv[e];
  for (int i = 0; i < m; ++i)
    if (!(dw[i] > 0.0)) return GKB_EINVAL;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 0) {
      CK(upload_csr<double>(c, m, wp, wc, wv, &c->csr64.W));
      CK(upload_csr<double>(c, m, ap, ac, av, &c->csr64.A));
      CK(upload_csr<double>(c, n, tp, tc, tv, &c->csr64.AT));
    } else {
      CK(upload_csr<float>(c, m, wp, wc, wv, &c->csr32.W));
      CK(upload_csr<float>(c, m, ap, ac, av, &c->csr32.A));
      CK(upload_csr<float>(c, n, tp, tc, tv, &c->csr32.AT));
    }
  }
  c->csr64.m = c->csr32.m = m;
  c->csr64.n = c->csr32.n = n;
  if (scaling == GKB_SCALE_CENTRAL) {
    std::vector<double> sw(m), sp(n, 0.0);
    for (int i = 0; i < m; ++i) sw[i] = 1.0 / std::sqrt(dw[i]);
    for (int i = 0; i < m; ++i)
      for (int e = ap[i]; e < ap[i + 1]; ++e) sp[ac[e]] += av[e] * av[e] / dw[i];
    for (int k = 0; k < n; ++k) {
      if (!(sp[k] > 0.0)) return GKB_EINVAL;  // an empty column of A
      sp[k] = 1.0 / std::sqrt(sp[k]);
    }
    double *sw64, *sp64;
    float *sw32, *sp32;
    CK(upload<double>(c, sw, &sw64));
    CK(upload<double>(c, sp, &sp64));
    CK(upload<float>(c, sw, &sw32));
    CK(upload<float>(c, sp, &sp32));
    c->csr64.sw = sw64;
    c->csr64.sp = sp64;
    c->csr32.sw = sw32;
    c->csr32.sp = sp32;
    c->csr_scaled = true;
    CK(c->mem.arr(&c->csr_gs, m));
    CK(c->mem.arr(&c->csr_rs, n));
  }
  CK(c->mem.arr(&c->csr_t64, n));
  CK(c->mem.arr(&c->csr_t32, n));
  c->op64 = Op<double>{};
  c->op64.g = G;
  c->op64.eta = eta;
  c->op32 = Op<float>{};
  c->op32.g = G;
  c->op32.eta = float(eta);
  c->fl0 = FaceLaunch{};
  c->fl0.nparts = c->fl0.gparts = vec_blocks(m);
  c->maxparts = std::max(vec_blocks(m), vec_blocks(n));
  for (int i = 0; i < kSlots; ++i) CK(c->mem.arr(&c->part[i], c->maxparts));
  CK(c->mem.arr(&c->dscal, 8));
  HIPCK(hipHostMalloc(reinterpret_cast<void**>(&c->hbuf), 4096, hipHostMallocDefault));
  double** fv[] = {&c->ghat, &c->w0, &c->u, &c->v, &c->Mv, &c->s, &c->y, &c->f, &c->rw, &c->dw};
  for (auto pp : fv) CK(c->mem.arr(pp, m));
  double** cv[] = {&c->b, &c->q, &c->d, &c->t, &c->rr, &c->dp};
  for (auto pp : cv) CK(c->mem.arr(pp, n));
  if (opt->refine_tol > 0.0) {
    CK(c->mem.arr(&c->wbest, m));
    CK(c->mem.arr(&c->pbest, n));
  }
  if (opt->method == GKB_METHOD_PRECOND) {
    const size_t pair = (size_t)m + n, R = (size_t)opt->outer_restart;
    CK(c->mem.arr(&c->ov, (R + 1) * pair));
    CK(c->mem.arr(&c->oz, R * pair));
    CK(c->mem.arr(&c->ozero, pair));
  }
  if (opt->precision == GKB_MIXED) CK(build_inner<float>(c, c->in32, c->coef32));
  else CK(build_inner<double>(c, c->in64, c->coef64));
  HIPCK(hipStreamSynchronize(c->cs));
  c->stats = gkb_stats_t{};
  return GKB_OK;
}

int validate_options(const gkb_options* o);

int validate(const gkb_grid* g, double eta, const gkb_options* o) {
  if (!g || (g->dim != 2 && g->dim != 3)) return GKB_EINVAL;
  if (!(g->h > 0.0) || !(eta >= 0.0) || !std::isfinite(eta)) return GKB_EINVAL;
  long nc = 1;
  for (int a = 0; a < g->dim; ++a) {
    if (g->n[a] < 2) return GKB_EINVAL;
    nc *= g->n[a];
  }
  if (nc > (1L << 30)) return GKB_EINVAL;
  bool all_nat = true;
  for (int s = 0; s < 2 * g->dim; ++s) {
    if (g->bc[s] != GKB_DIRICHLET && g->bc[s] != GKB_NATURAL) return GKB_EINVAL;
    all_nat = all_nat && g->bc[s] == GKB_NATURAL;
  }
  if (all_nat) return GKB_EINVAL;
  if (g->pin_cell < -1 || g->pin_cell >= nc) return GKB_EINVAL;
  return validate_options(o);
}

int validate_options(const gkb_options* o) {
  if (o->precision != GKB_FP64 && o->precision != GKB_MIXED) return GKB_EINVAL;
  if (o->inner < 0 || o->inner > 2) return GKB_EINVAL;
  if (o->nu_pre < 0 || o->nu_post < 0 || o->nu_pre + o->nu_post < 1) return GKB_EINVAL;
  if (o->inner_maxit < 1 || o->maxit < 1 || o->max_sweeps < 1) return GKB_EINVAL;
  if (o->check_every < 1 || o->stencil < 0 || o->stencil > 1) return GKB_EINVAL;
  if (o->smoother != GKB_SMOOTH_JACOBI && o->smoother != GKB_SMOOTH_HYBRID) return GKB_EINVAL;
  if (o->krylov != GKB_KRYLOV_CG && o->krylov != GKB_KRYLOV_FGMRES) return GKB_EINVAL;
  if (o->fgmres_restart < 1 || o->fgmres_restart > kMaxRestart) return GKB_EINVAL;
  if (o->method != GKB_METHOD_SOLVER && o->method != GKB_METHOD_PRECOND) return GKB_EINVAL;
  if (o->method == GKB_METHOD_PRECOND && !(o->refine_tol > 0.0)) return GKB_EINVAL;
  if (o->outer_restart < 1 || o->outer_restart > kMaxOuterRestart) return GKB_EINVAL;
  if (!std::isfinite(o->learned_min_gain)) return GKB_EINVAL;
  if (o->mg_transfer < GKB_TRANSFER_AUTO || o->mg_transfer > GKB_TRANSFER_SMOOTH) return GKB_EINVAL;
  if (o->cnn_weights && o->inner != GKB_INNER_LEARNED) return GKB_EINVAL;
  return GKB_OK;
}

}  // namespace

// ------------------------------------------------------------------ C-ABI

extern "C" {

void gkb_default_options(gkb_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->precision = GKB_FP64;
  o->inner = GKB_INNER_MG;
  o->mg_levels = 0;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->inner_tol = 1e-10;
  o->inner_maxit = 10000;
  o->maxit = 500;
  o->refine_tol = 0.0;
  o->max_sweeps = 10;
  o->check_every = 8;
  o->use_graphs = 1;
  o->stencil = 0;
  o->smoother = GKB_SMOOTH_JACOBI;
  o->hip_stream = nullptr;
  o->max_workspace_bytes = 0;
  o->krylov = GKB_KRYLOV_CG;
  o->fgmres_restart = 30;
  o->method = GKB_METHOD_SOLVER;
  o->outer_restart = 10;
  o->cnn_weights = nullptr;
  o->learned_min_gain = 0.05;
  o->mg_transfer = GKB_TRANSFER_AUTO;
}

int gkb_setup(const gkb_grid* grid, const double* viscosity, double eta, const gkb_options* opt,
              gkb_ctx** out) {
  if (!out) return GKB_EINVAL;
  *out = nullptr;
  gkb_options o;
  if (opt) o = *opt;
  else gkb_default_options(&o);
  int rc = validate(grid, eta, &o);
  if (rc) return rc;
  if (viscosity) {
    long nc = (long)grid->n[0] * grid->n[1] * (grid->dim == 3 ? grid->n[2] : 1);
    for (long i = 0; i < nc; ++i)
      if (!(viscosity[i] > 0.0) || !std::isfinite(viscosity[i])) return GKB_EINVAL;
  }
  gkb_ctx* c = new (std::nothrow) gkb_ctx();
  if (!c) return GKB_ENOMEM;
  rc = setup_impl(c, grid, viscosity, eta, &o);
  if (rc < 0) {
    gkb_destroy(c);
    return rc;
  }
  *out = c;
  return GKB_OK;
}

int gkb_setup_csr(const gkb_csr* sys, double eta, int scaling, const gkb_options* opt,
                  gkb_ctx** out) {
  if (!out) return GKB_EINVAL;
  *out = nullptr;
  if (!sys || !(eta >= 0.0) || !std::isfinite(eta)) return GKB_EINVAL;
  if (scaling != GKB_SCALE_NONE && scaling != GKB_SCALE_CENTRAL) return GKB_EINVAL;
  gkb_options o;
  if (opt) o = *opt;
  else gkb_default_options(&o);
  o.inner = opt ? o.inner : GKB_INNER_JACOBI;  // the default multigrid needs a grid
  int rc = validate_options(&o);
  if (rc) return rc;
  if (o.inner != GKB_INNER_JACOBI || o.cnn_weights) return GKB_EINVAL;
  if (!csr_valid(sys->m, sys->m, sys->w_rowptr, sys->w_col, sys->w_val) ||
      !csr_valid(sys->m, sys->n, sys->a_rowptr, sys->a_col, sys->a_val))
    return GKB_EINVAL;
  gkb_ctx* c = new (std::nothrow) gkb_ctx();
  if (!c) return GKB_ENOMEM;
  rc = setup_csr_impl(c, sys, eta, scaling, &o);
  if (rc < 0) {
    gkb_destroy(c);
    return rc;
  }
  *out = c;
  return GKB_OK;
}

int gkb_solve(gkb_ctx* c, const double* g, const double* r, double tol, int delay, double* w,
              double* p, int* iterations, double* error_estimate) {
  if (!c || !g || !r || !w || !p || delay < 1) return GKB_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  HIPCK(hipEventRecord(c->ev, c->us));
  HIPCK(hipStreamWaitEvent(c->cs, c->ev, 0));
  c->stats.sweeps = 0;
  c->stats.outer_iterations = 0;
  c->stats.inner_iterations = 0;
  c->stats.inner_solves = 0;
  c->stats.fallbacks = 0;
  c->stats.learned_solves = 0;
  c->stats.residual = -1.0;
  c->stats.learned_gain = -1.0;
  c->stats.learned_fallback_reason = 0;
  c->stats.learned_fallback_iteration = 0;
  c->stats.outer_krylov_iterations = 0;
  learned_reset(c->learned);
  if (c->csr_scaled) {
    // the iteration runs on the centrally scaled system: g' = D^-1/2 g,
    // r' = R^-1/2 r; the solution is scaled back at the end
    k_scale<<<vec_blocks(c->g.m_full), kBlock, 0, c->cs>>>(c->g.m_full, c->csr64.sw, g, c->csr_gs);
    k_scale<<<vec_blocks(c->g.n_cells), kBlock, 0, c->cs>>>(c->g.n_cells, c->csr64.sp, r, c->csr_rs);
    g = c->csr_gs;
    r = c->csr_rs;
  }
  int K = 0, rc;
  double est = 0.0;
  if (c->opt.method == GKB_METHOD_PRECOND) {
    rc = precond_solve(c, g, r, tol, delay, w, p, &K, &est);
  } else if (c->opt.refine_tol <= 0.0) {
    rc = gkb_run(c, g, r, tol, delay, w, p, &K, &est);
    c->stats.sweeps = 1;
  } else {
    // defect correction: (w, p) += GKB(res) until the FP64 residual is small
    const int m = c->g.m_full, nc = c->g.n_cells;
    k_fill<double><<<vec_blocks(m), kBlock, 0, c->cs>>>(m, 0.0, w);
    k_fill<double><<<vec_blocks(nc), kBlock, 0, c->cs>>>(nc, 0.0, p);
    double norms[4];
    // best iterate so far: a sweep may raise the residual before later ones
    // converge, but three sweeps without a new best (or growth by 1e3) mean
    // the inner solves are too inexact for the correction to converge
    double best = HUGE_VAL;
    int since_best = 0;
    auto restore_best = [&]() {
      k_cast<double, double><<<vec_blocks(m), kBlock, 0, c->cs>>>(m, c->wbest, w);
      k_cast<double, double><<<vec_blocks(nc), kBlock, 0, c->cs>>>(nc, c->pbest, p);
      c->stats.residual = best;
    };
    rc = GKB_MAXIT;
    for (int sw = 0; sw <= c->opt.max_sweeps; ++sw) {
      int r2 = residual_impl(c, g, r, w, p, c->rw, c->rr, norms);
      if (r2 < 0) return r2;
      const double rel = norms[3] > 0 ? norms[0] / norms[3] : 0.0;
      c->stats.residual = rel;
      if (!std::isfinite(rel)) {
        if (sw > 0) restore_best();
        rc = GKB_ENAN;
        break;
      }
      if (rel < best) {
        best = rel;
        since_best = 0;
        k_cast<double, double><<<vec_blocks(m), kBlock, 0, c->cs>>>(m, w, c->wbest);
        k_cast<double, double><<<vec_blocks(nc), kBlock, 0, c->cs>>>(nc, p, c->pbest);
      } else {
        ++since_best;
      }
      if (rel <= c->opt.refine_tol) {
        rc = GKB_OK;
        break;
      }
      if (since_best >= 3 || rel > 1e3 * best || sw == c->opt.max_sweeps) {
        if (rel > best) restore_best();
        break;
      }
      int r3 = gkb_run(c, c->rw, c->rr, tol, delay, c->dw, c->dp, &K, &est);
      c->stats.sweeps += 1;
      if (r3 < 0) {
        rc = r3;
        break;
      }
      k_axpby<<<vec_blocks(m), kBlock, 0, c->cs>>>(m, 1.0, c->dw, 1.0, w);
      k_axpby<<<vec_blocks(nc), kBlock, 0, c->cs>>>(nc, 1.0, c->dp, 1.0, p);
    }
  }
  if (c->csr_scaled) {
    k_scale<<<vec_blocks(c->g.m_full), kBlock, 0, c->cs>>>(c->g.m_full, c->csr64.sw, w, w);
    k_scale<<<vec_blocks(c->g.n_cells), kBlock, 0, c->cs>>>(c->g.n_cells, c->csr64.sp, p, p);
  }
  HIPCK(hipStreamSynchronize(c->cs));
  c->stats.seconds_solve =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (iterations) *iterations = K;
  if (error_estimate) *error_estimate = est;
  return rc;
}

int gkb_stats(const gkb_ctx* c, gkb_stats_t* out) {
  if (!c || !out) return GKB_EINVAL;
  *out = c->stats;
  out->workspace_bytes = c->mem.bytes;
  out->mg_levels = c->L;
  for (int l = 0; l < c->L && l < 16; ++l) out->omega[l] = c->omega[l];
  for (int l = 0; l < (int)c->omega_e.size() && l < 16; ++l) out->omega_edge[l] = c->omega_e[l];
  out->mg_transfer = c->smooth_transfer ? GKB_TRANSFER_SMOOTH : GKB_TRANSFER_DIV;
  return GKB_OK;
}

int gkb_sizes(const gkb_ctx* c, long* m_full, long* n_cells, long* m_unknown, long* n_unknown) {
  if (!c) return GKB_EINVAL;
  const Grid& g = c->g;
  if (m_full) *m_full = g.m_full;
  if (n_cells) *n_cells = g.n_cells;
  if (c->csr) {
    if (m_unknown) *m_unknown = g.m_full;
    if (n_unknown) *n_unknown = g.n_cells;
    return GKB_OK;
  }
  long mu = 0;
  for (int cc = 0; cc < g.dim; ++cc) {
    long plane = (long)g.ext[cc][0] * g.ext[cc][1] * g.ext[cc][2] / g.ext[cc][cc];
    long cnt = g.ext[cc][cc];
    if (g.bc[2 * cc] == GKB_DIRICHLET) --cnt;
    if (g.bc[2 * cc + 1] == GKB_DIRICHLET) --cnt;
    mu += plane * cnt;
  }
  if (m_unknown) *m_unknown = mu;
  if (n_unknown) *n_unknown = g.n_cells - (g.pin >= 0 ? 1 : 0);
  return GKB_OK;
}

const char* gkb_strerror(int code) {
  switch (code) {
    case GKB_OK: return "ok";
    case GKB_MAXIT: return "maximum number of GKB iterations reached";
    case GKB_EINVAL: return "invalid argument";
    case GKB_ENOMEM: return "out of memory or workspace cap exceeded";
    case GKB_EHIP: return "HIP runtime error";
    case GKB_ENAN: return "non-finite value in the iteration";
    case GKB_EINNER: return "inner solve did not converge within inner_maxit";
    default: return "unknown error code";
  }
}

void gkb_destroy(gkb_ctx* c) {
  if (!c) return;
  if (c->cs) (void)hipStreamSynchronize(c->cs);
  if (c->in64.graph) (void)hipGraphExecDestroy(c->in64.graph);
  if (c->in32.graph) (void)hipGraphExecDestroy(c->in32.graph);
  if (c->in64.graph_fcg) (void)hipGraphExecDestroy(c->in64.graph_fcg);
  if (c->in32.graph_fcg) (void)hipGraphExecDestroy(c->in32.graph_fcg);
  if (c->in64.graph_gm) (void)hipGraphExecDestroy(c->in64.graph_gm);
  if (c->in32.graph_gm) (void)hipGraphExecDestroy(c->in32.graph_gm);
  if (c->learned) learned_destroy(c);
  if (c->owned_net) gkb_cnn_destroy(c->owned_net);
  c->mem.release();
  if (c->hbuf) (void)hipHostFree(c->hbuf);
  if (c->ev) (void)hipEventDestroy(c->ev);
  if (c->cs) (void)hipStreamDestroy(c->cs);
  delete c;
}

int gkb_apply(gkb_ctx* c, int op, int precision, const void* x, void* y) {
  if (!c || !y || (op != GKB_OP_DIAG && !x)) return GKB_EINVAL;
  HIPCK(hipEventRecord(c->ev, c->us));
  HIPCK(hipStreamWaitEvent(c->cs, c->ev, 0));
  const Grid& G = c->g;
  if (precision == GKB_FP64) {
    const double* xd = static_cast<const double*>(x);
    double* yd = static_cast<double*>(y);
    Op<double> o = c->op64;
    switch (op) {
      case GKB_OP_W: o.eta = 0.0; face_op<double, kApply>(c, o, c->fl0, xd, nullptr, yd, 0.0, nullptr, nullptr); break;
      case GKB_OP_M: face_op<double, kApply>(c, o, c->fl0, xd, nullptr, yd, 0.0, nullptr, nullptr); break;
      case GKB_OP_DIAG: face_op<double, kDiag>(c, o, c->fl0, nullptr, nullptr, yd, 0.0, nullptr, nullptr); break;
      case GKB_OP_A: grad_axpy(c, xd, nullptr, 1.0, 0.0, yd); break;
      case GKB_OP_AT: div_axpy<double>(c, G, xd, nullptr, 1.0, 0.0, yd, nullptr, nullptr); break;
      default: return GKB_EINVAL;
    }
  } else if (precision == GKB_MIXED) {
    const float* xf = static_cast<const float*>(x);
    float* yf = static_cast<float*>(y);
    Op<float> o = c->op32;
    switch (op) {
      case GKB_OP_W: o.eta = 0.0f; face_op<float, kApply>(c, o, c->fl0, xf, nullptr, yf, 0.0f, nullptr, nullptr); break;
      case GKB_OP_M: face_op<float, kApply>(c, o, c->fl0, xf, nullptr, yf, 0.0f, nullptr, nullptr); break;
      case GKB_OP_DIAG: face_op<float, kDiag>(c, o, c->fl0, nullptr, nullptr, yf, 0.0f, nullptr, nullptr); break;
      case GKB_OP_AT: div_axpy<float>(c, G, xf, nullptr, 1.0, 0.0, yf, nullptr, nullptr); break;
      default: return GKB_EINVAL;
    }
  } else {
    return GKB_EINVAL;
  }
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(c->cs));
  return GKB_OK;
}

int gkb_precondition(gkb_ctx* c, int precision, const void* r, void* z) {
  if (!c || !r || !z) return GKB_EINVAL;
  HIPCK(hipEventRecord(c->ev, c->us));
  HIPCK(hipStreamWaitEvent(c->cs, c->ev, 0));
  const int m = c->g.m_full;
  if (precision == GKB_FP64) {
    if (!c->in64.ready) return GKB_EINVAL;
    Inner<double>& in = c->in64;
    if (c->opt.inner == GKB_INNER_JACOBI)
      k_pcg_p0<double><<<vec_blocks(m), kBlock, 0, c->cs>>>(m, in.dinv, static_cast<const double*>(r),
                                                            static_cast<double*>(z), in.q, c->part[0]);
    else
      vcycle<double>(c, in, 0, static_cast<const double*>(r), static_cast<double*>(z), nullptr, nullptr);
  } else if (precision == GKB_MIXED) {
    if (!c->in32.ready) return GKB_EINVAL;
    Inner<float>& in = c->in32;
    if (c->opt.inner == GKB_INNER_JACOBI)
      k_pcg_p0<float><<<vec_blocks(m), kBlock, 0, c->cs>>>(m, in.dinv, static_cast<const float*>(r),
                                                           static_cast<float*>(z), in.q, c->part[0]);
    else
      vcycle<float>(c, in, 0, static_cast<const float*>(r), static_cast<float*>(z), nullptr, nullptr);
  } else {
    return GKB_EINVAL;
  }
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(c->cs));
  return GKB_OK;
}

int gkb_inner_solve(gkb_ctx* c, const double* f, double* x, double tol, int* iterations) {
  if (!c || !f || !x) return GKB_EINVAL;
  HIPCK(hipEventRecord(c->ev, c->us));
  HIPCK(hipStreamWaitEvent(c->cs, c->ev, 0));
  int rc = inner_solve_any(c, f, x, tol > 0 ? tol : c->opt.inner_tol, iterations);
  HIPCK(hipStreamSynchronize(c->cs));
  return rc;
}

int gkb_residual(gkb_ctx* c, const double* g, const double* r, const double* w, const double* p,
                 double* res_w, double* res_r, double* norms) {
  if (!c || !g || !r || !w || !p || !norms) return GKB_EINVAL;
  HIPCK(hipEventRecord(c->ev, c->us));
  HIPCK(hipStreamWaitEvent(c->cs, c->ev, 0));
  return residual_impl(c, g, r, w, p, res_w, res_r, norms, true);
}

}  // extern "C"

namespace {
template <typename T>
int time_kernel_impl(gkb_ctx* c, Inner<T>& in, int kernel, int reps, double* avg_ms) {
  if (!in.ready || reps < 1) return GKB_EINVAL;
  Level<T>& L = in.lv[0];
  if ((kernel == GKB_KERNEL_SMOOTH_PROLONG || kernel == GKB_KERNEL_SMOOTH_ZERO) &&
      (!L.fl.tiled || c->L < 2))
    return GKB_EINVAL;
  if (kernel == GKB_KERNEL_SMOOTH_ZERO && L.op.mu != nullptr) return GKB_EINVAL;
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  auto one = [&]() {
    if (kernel == GKB_KERNEL_SMOOTH)
      face_op<T, kJacobi>(c, L.op, L.fl, in.z, in.r, L.t, T(L.omega), nullptr, nullptr);
    else if (kernel == GKB_KERNEL_SMOOTH_PROLONG)
      face_op<T, kJacobiP>(c, L.op, L.fl, in.z, in.r, L.t, T(L.omega), nullptr, nullptr,
                           in.lv[1].x, &in.lv[1].g);
    else if (kernel == GKB_KERNEL_SMOOTH_ZERO)
      face_op<T, kJacobiZ>(c, L.op, L.fl, in.r, in.r, L.t, T(L.omega), nullptr, nullptr);
    else if (kernel == GKB_KERNEL_APPLY)
      face_op<T, kApplyDot>(c, L.op, L.fl, in.p, nullptr, in.q, T(0), c->part[0], nullptr);
    else
      face_op<T, kResid>(c, L.op, L.fl, in.z, in.r, L.rb, T(0), nullptr, nullptr);
  };
  // the launches are captured into one HIP graph and replayed, as the solver
  // replays its PCG iterations, so the per-launch time is the kernel's
  // duration plus the graph's (small) gap between nodes
  one();  // warm-up launch
  hipGraph_t gr;
  hipGraphExec_t ge = nullptr;
  HIPCK(hipStreamBeginCapture(c->cs, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < reps; ++i) one();
  HIPCK(hipStreamEndCapture(c->cs, &gr));
  const hipError_t ie = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  HIPCK(ie);
  HIPCK(hipGraphLaunch(ge, c->cs));  // warm-up replay
  HIPCK(hipEventRecord(e0, c->cs));
  HIPCK(hipGraphLaunch(ge, c->cs));
  HIPCK(hipEventRecord(e1, c->cs));
  HIPCK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCK(hipEventElapsedTime(&ms, e0, e1));
  *avg_ms = double(ms) / reps;
  (void)hipGraphExecDestroy(ge);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return GKB_OK;
}
}  // namespace

extern "C" int gkb_time_kernel(gkb_ctx* c, int kernel, int reps, double* avg_ms) {
  if (!c || !avg_ms || kernel < 0 || kernel > 4 || c->opt.inner == GKB_INNER_JACOBI) return GKB_EINVAL;
  if (c->opt.precision == GKB_MIXED) return time_kernel_impl<float>(c, c->in32, kernel, reps, avg_ms);
  return time_kernel_impl<double>(c, c->in64, kernel, reps, avg_ms);
}

#include "noalloc.hpp"
