// Allocation-free variant of gkb_residual (included by gkb.hip after the
// C-ABI): the FP64 saddle residual for mu = 1 without a solver context, for
// callers that cannot allocate device memory.
#pragma once
#include <mutex>

// gkb_residual_noalloc: the saddle residual of gkb_residual for mu = 1
// without a context.  Its reduction partials live in `scratch`, a fixed
// device array (one copy per GPU, held until the process ends); the host
// reaches it only through the address hipGetSymbolAddress returns for the
// current device, taken once per device.
namespace {

constexpr int kScratchParts = 65536;  // partials per reduction (4 reductions)
constexpr int kScratchDoubles = 4 * kScratchParts + 8;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {nullptr};

// the current device's copy of `scratch` (its address, not the host-side
// name), looked up on the first call on each device
int scratch_on_current_device(double** out) {
  int dev = -1;
  HIPCK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return GKB_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return GKB_EHIP;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return GKB_OK;
}

}  // namespace

extern "C" int gkb_residual_noalloc(const gkb_grid* grid, const double* g, const double* r,
                                    const double* w, const double* p, double* res_w,
                                    double* res_r, double* norms, void* hip_stream) {
  if (!grid || !g || !r || !w || !p || !res_r || !norms) return GKB_EINVAL;
  gkb_options o;
  gkb_default_options(&o);
  CK(validate(grid, 0.0, &o));
  const int n[3] = {grid->n[0], grid->n[1], grid->dim == 3 ? grid->n[2] : 1};
  const Grid G = make_grid(grid->dim, n, grid->h, grid->bc, grid->pin_cell);
  // the generic face kernel's launch, the same as gkb_residual's, so both
  // reduce in the same order
  const FaceLaunch fl = face_launch(G, 4, 1);
  const int pw = fl.gparts, pc = cell_parts(G);
  if (pw > kScratchParts || pc > kScratchParts) return GKB_EINVAL;  // grid too large
  double* sc = nullptr;
  CK(scratch_on_current_device(&sc));
  double *p_rr = sc, *p_gg = sc + kScratchParts, *p_tt = sc + 2 * kScratchParts,
         *p_zz = sc + 3 * kScratchParts, *sums = sc + 4 * kScratchParts;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Op<double> opW{};
  opW.g = G;
  opW.eta = 0.0;
  opW.ih2 = 1.0 / (G.h * G.h);
  opW.ih = 1.0 / G.h;
  if (G.dim == 2)
    k_resid_w<2, false><<<fl.grid, kBlock, 0, s>>>(opW, g, w, p, res_w, fl.kz, fl.zchunks, p_rr, p_gg);
  else
    k_resid_w<3, false><<<fl.grid, kBlock, 0, s>>>(opW, g, w, p, res_w, fl.kz, fl.zchunks, p_rr, p_gg);
  // res_r = r - A^T w (required: the cell residual is formed in it)
  double* t_out = res_r;
  if (G.dim == 2)
    k_div_axpy<double, 2><<<cell_grid(G), kBlock, 0, s>>>(G, w, r, -1.0, 1.0, t_out, p_tt, p_zz);
  else
    k_div_axpy<double, 3><<<cell_grid(G), kBlock, 0, s>>>(G, w, r, -1.0, 1.0, t_out, p_tt, p_zz);
  k_sum_partials<<<1, kFinal, 0, s>>>(p_rr, pw, sums + 0);
  k_sum_partials<<<1, kFinal, 0, s>>>(p_gg, pw, sums + 1);
  k_sum_partials<<<1, kFinal, 0, s>>>(p_tt, pc, sums + 2);
  k_sum_partials<<<1, kFinal, 0, s>>>(p_zz, pc, sums + 3);
  HIPCK(hipGetLastError());
  double h[4];
  HIPCK(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  norms[0] = std::sqrt(h[0] + h[2]);
  norms[1] = std::sqrt(h[0]);
  norms[2] = std::sqrt(h[2]);
  norms[3] = std::sqrt(h[1] + h[3]);
  return GKB_OK;
}

#include "learned_impl.hpp"
