// Convolutional preconditioner network on gfx950 (see include/gkb_cnn.h).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x16_bf16: a wave64
// computes 16 output points x 16 output channels; the GEMM K dimension runs
// over taps x input channels, 16 deep per MFMA: one tap of 16 channels, two
// taps of 8 or four taps of 4 (a layer reads only the channel group its
// input fills, so 8- and 4-channel inputs take 2x and 4x fewer MFMAs and
// gathered bytes).
// Activations are channels-last BF16 padded to 16 channels (32 bytes per
// point), so the A fragment of a lane (4 consecutive channels of one point)
// is one 8-byte load; the 3x3(x3) weights of a layer sit in LDS in the
// B-fragment order [tap][c_out][c_in].  The weight gradient is a GEMM over
// points (K = points) with one accumulator tile per tap; blocks write FP32
// partials that a second kernel sums in a fixed order (deterministic).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/gkb_cnn.h"

namespace gkb {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kCP = 16;        // padded channel count
constexpr int kMaxLayers = 8;

__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return uint16_t(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

struct CnnGeom {
  int nx, ny, nz, batch;
  long P;  // nx * ny * nz * batch
};

__device__ __forceinline__ void tap_off(int t, int dim, int& dx, int& dy, int& dz) {
  dx = t % 3 - 1;
  dy = (t / 3) % 3 - 1;
  dz = dim == 3 ? t / 9 - 1 : 0;
}

// neighbour of point p (coordinates i, j, k in one grid) at offset; -1 if
// outside the grid
__device__ __forceinline__ long nb_index(const CnnGeom& g, long p, int i, int j, int k, int dx,
                                         int dy, int dz) {
  const int ii = i + dx, jj = j + dy, kk = k + dz;
  if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) return -1;
  return p + dx + (long)dy * g.nx + (long)dz * g.nx * g.ny;
}

// coordinates of point p in its grid, in 32-bit arithmetic (every network
// call keeps batch * points below 2^31)
__device__ __forceinline__ void coords(const CnnGeom& g, long p, int& i, int& j, int& k) {
  const unsigned q = unsigned(p), nx = unsigned(g.nx), ny = unsigned(g.ny);
  const unsigned r = q / nx, s = r / ny;
  i = int(q - r * nx);
  j = int(r - s * ny);
  k = int(s % unsigned(g.nz));
}

enum ConvOut { kOutReluBf16 = 0, kOutF32 = 1, kOutMaskBf16 = 2 };

// Blocks for a convolution over P points: each block stages the layer's
// weights in LDS once and then takes groups of 64 points (16 per wave) in a
// grid-stride loop, so the weight staging is paid per block, not per group.
// At most 8192 blocks: a 64^3 x 2 training batch keeps one group per block
// (a 2048-block cap, four groups per block, made its gradient layers 25 %
// slower: each wave waits on its loads group after group), and a 128^3
// inference pass takes four groups per block.
inline int conv_blocks(long P) {
  const long groups = (P + 63) / 64;
  return int(groups < 8192 ? groups : 8192);
}

// out[p][n] = bias[n] + sum_tap sum_c in[p + off(tap)][c] * w[tap][n][c],
// the input channels c < CG (16, 8 or 4; the padded channels above are zero)
template <int DIM, int OUT, int CG = kCP>
__global__ __launch_bounds__(256) void k_conv(CnnGeom g, const uint16_t* __restrict__ in,
                                              const uint16_t* __restrict__ w,
                                              const float* __restrict__ bias, void* __restrict__ out,
                                              const uint16_t* __restrict__ mask,
                                              const int* __restrict__ skip1 = nullptr,
                                              const int* __restrict__ skip2 = nullptr) {
  constexpr int TAPS = DIM == 2 ? 9 : 27;
  static_assert(CG == 16 || CG == 8 || CG == 4, "channel group");
  constexpr int TPM = kCP / CG;  // taps per MFMA
  // device-side switches (solve converged / learned correction disabled)
  if ((skip1 && *skip1) || (skip2 && *skip2)) return;
  __shared__ uint16_t sw[TAPS * 256];
  for (int e = threadIdx.x; e < TAPS * 256; e += 256) sw[e] = w[e];
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = lane & 15, kg = lane >> 4;
  // the lane's four K values: tap t + tsub, channels c0 .. c0 + 3
  const int tsub = CG == 16 ? 0 : (CG == 8 ? kg >> 1 : kg);
  const int c0 = CG == 16 ? 4 * kg : (CG == 8 ? 4 * (kg & 1) : 0);
  for (long base = (long)blockIdx.x * 64; base < g.P; base += (long)gridDim.x * 64) {
    const long p0 = base + wv * 16;
    if (p0 >= g.P) break;
    const long p = p0 + m;
    const bool valid = p < g.P;
    int i = 0, j = 0, k = 0;
    if (valid) coords(g, p, i, j, k);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t0 = 0; t0 < TAPS; t0 += TPM) {
      const int t = t0 + tsub;
      int dx, dy, dz;
      tap_off(t, DIM, dx, dy, dz);
      bf16x4 a = {0, 0, 0, 0}, b = {0, 0, 0, 0};
      if (t < TAPS) {  // the last group of a layer may run past the taps
        if (valid) {
          const long q = nb_index(g, p, i, j, k, dx, dy, dz);
          if (q >= 0) a = *reinterpret_cast<const bf16x4*>(in + q * kCP + c0);
        }
        b = *reinterpret_cast<const bf16x4*>(sw + t * 256 + m * 16 + c0);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    // acc[q] = D[row 4kg+q][col m]: point p0 + 4kg + q, channel m
    const float bm = bias ? bias[m] : 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long pq = p0 + 4 * kg + q;
      if (pq >= g.P) continue;
      float v = acc[q] + bm;
      if (OUT == kOutReluBf16) {
        static_cast<uint16_t*>(out)[pq * kCP + m] = f2bf(v > 0.f ? v : 0.f);
      } else if (OUT == kOutF32) {
        static_cast<float*>(out)[pq * kCP + m] = v;
      } else {
        const uint16_t h = mask[pq * kCP + m];
        const bool pos = h != 0 && (h & 0x8000u) == 0;
        static_cast<uint16_t*>(out)[pq * kCP + m] = f2bf(pos ? v : 0.f);
      }
    }
  }
}

// Launch k_conv with the smallest channel group that holds the input's
// cin channels.
template <int DIM, int OUT>
void launch_conv(int cin, int blocks, hipStream_t s, const CnnGeom& g, const uint16_t* in,
                 const uint16_t* w, const float* bias, void* out, const uint16_t* mask,
                 const int* skip1 = nullptr, const int* skip2 = nullptr) {
  if (cin <= 4)
    k_conv<DIM, OUT, 4><<<blocks, 256, 0, s>>>(g, in, w, bias, out, mask, skip1, skip2);
  else if (cin <= 8)
    k_conv<DIM, OUT, 8><<<blocks, 256, 0, s>>>(g, in, w, bias, out, mask, skip1, skip2);
  else
    k_conv<DIM, OUT, 16><<<blocks, 256, 0, s>>>(g, in, w, bias, out, mask, skip1, skip2);
}

// Weight / bias gradient partials of one layer: for every tap
//   dW[tap][ci][co] = sum_p act[p + off(tap)][ci] * dz[p][co],  db[co] = sum_p dz[p][co]
// Each block covers a strided set of 16-point chunks and writes TAPS*256+16
// FP32 partials.  The 16 rows of an MFMA tile are (tap, ci) pairs: one tap
// of 16 input channels, two taps of 8 or four of 4 (CG), so a layer with
// few input channels needs fewer tiles.
template <int DIM, int CG = kCP>
__global__ __launch_bounds__(256) void k_wgrad(CnnGeom g, const uint16_t* __restrict__ act,
                                               const uint16_t* __restrict__ dz,
                                               float* __restrict__ part) {
  constexpr int TAPS = DIM == 2 ? 9 : 27;
  constexpr int NP = TAPS * 256 + 16;
  static_assert(CG == 16 || CG == 8 || CG == 4, "channel group");
  constexpr int TPM = kCP / CG;                 // taps per tile
  constexpr int NT = (TAPS + TPM - 1) / TPM;    // tiles
  __shared__ float red[NP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = lane & 15, kg = lane >> 4;
  // the lane's A row m: tap t * TPM + msub, input channel mc
  const int msub = m / CG, mc = m % CG;
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float db = 0.f;
  const long nchunks = (g.P + 15) / 16;
  const long nw = (long)gridDim.x * 4;
  for (long c = (long)blockIdx.x * 4 + wv; c < nchunks; c += nw) {
    const long p0 = c * 16;
    bf16x4 b;
    long pq[4];
    int ci[4], cj[4], ck[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      pq[q] = p0 + 4 * kg + q;
      if (pq[q] < g.P) {
        b[q] = (short)dz[pq[q] * kCP + m];
        coords(g, pq[q], ci[q], cj[q], ck[q]);
      } else {
        b[q] = 0;
        ci[q] = cj[q] = ck[q] = 0;
      }
      db += bf2f((uint16_t)b[q]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int tap = t * TPM + msub;
      int dx, dy, dzz;
      tap_off(tap, DIM, dx, dy, dzz);
      bf16x4 a;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = 0;
        if (tap < TAPS && pq[q] < g.P) {
          const long n = nb_index(g, pq[q], ci[q], cj[q], ck[q], dx, dy, dzz);
          if (n >= 0) a[q] = (short)act[n * kCP + mc];
        }
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
  __shared__ float dbs[256];
  for (int e = threadIdx.x; e < NP; e += 256) red[e] = 0.f;
  dbs[threadIdx.x] = db;  // slot (wave, kg, m)
  __syncthreads();
  // waves add their tiles in a fixed order: D[row 4kg+q][co = m], row =
  // (tap t * TPM + row / CG, ci = row % CG); every barrier below is reached
  // by all waves
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 4 * kg + q, tap = t * TPM + row / CG;
          if (tap < TAPS) red[tap * 256 + (row % CG) * 16 + m] += acc[t][q];
        }
    }
    __syncthreads();
  }
  if (threadIdx.x < 16) {
    float s = 0.f;
    for (int e = 0; e < 16; ++e) s += dbs[(e >> 2) * 64 + (e & 3) * 16 + threadIdx.x];
    red[TAPS * 256 + threadIdx.x] = s;
  }
  __syncthreads();
  float* dst = part + (size_t)blockIdx.x * NP;
  for (int e = threadIdx.x; e < NP; e += 256) dst[e] = red[e];
}

// Sum the block partials in a fixed order: a block takes 16 consecutive
// outputs; its 16 thread groups sum the partials b = g, g + 16, ... of
// them, and the 16 group sums are added in order.
constexpr int kRedOut = 16;
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int nblk,
                                                      int np, float* __restrict__ out) {
  const int o = threadIdx.x % kRedOut, grp = threadIdx.x / kRedOut;
  const int e = blockIdx.x * kRedOut + o;
  float s = 0.f;
  if (e < np)
    for (int b = grp; b < nblk; b += 256 / kRedOut) s += part[(size_t)b * np + e];
  __shared__ float sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (grp == 0 && e < np) {
    float t = 0.f;
    for (int g = 0; g < 256 / kRedOut; ++g) t += sh[g * kRedOut + o];
    out[e] = t;
  }
}

// padded gradient [taps][ci][co] + db[co] -> flat layer layout W[tap][ci][co], b[co]
__global__ __launch_bounds__(256) void k_grad_flat(const float* __restrict__ pad, int taps, int cin,
                                                   int cout, float* __restrict__ flat) {
  const int n = taps * cin * cout + cout;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    if (e < taps * cin * cout) {
      const int co = e % cout, ci = (e / cout) % cin, t = e / (cout * cin);
      flat[e] = pad[t * 256 + ci * 16 + co];
    } else {
      flat[e] = pad[taps * 256 + (e - taps * cin * cout)];
    }
  }
}

// flat FP32 layer parameters -> BF16 forward weights wf[t][co][ci], dgrad
// weights wd[t][ci][co] taken from the mirrored tap, FP32 bias[16]
__global__ __launch_bounds__(256) void k_pack_weights(const float* __restrict__ flat, int taps,
                                                      int cin, int cout, uint16_t* __restrict__ wf,
                                                      uint16_t* __restrict__ wd,
                                                      float* __restrict__ bias) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < taps * 256; e += gridDim.x * 256) {
    const int t = e / 256, a = (e / 16) % 16, c = e % 16;
    // wf[t][a = co][c = ci]
    float vf = (a < cout && c < cin) ? flat[(t * cin + c) * cout + a] : 0.f;
    wf[e] = f2bf(vf);
    // wd[t][a = ci (output of the adjoint)][c = co] = W[taps-1-t][ci][co]
    const int tm = taps - 1 - t;
    float vd = (a < cin && c < cout) ? flat[(tm * cin + a) * cout + c] : 0.f;
    wd[e] = f2bf(vd);
  }
  if (blockIdx.x == 0 && threadIdx.x < 16)
    bias[threadIdx.x] = threadIdx.x < cout ? flat[taps * cin * cout + threadIdx.x] : 0.f;
}

// FP32 [P][c] -> BF16 [P][16] (zero padding)
__global__ __launch_bounds__(256) void k_to_act(long P, int c, const float* __restrict__ x,
                                                uint16_t* __restrict__ a) {
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < P * kCP; e += (long)gridDim.x * 256) {
    const long p = e / kCP;
    const int ch = int(e % kCP);
    a[e] = f2bf(ch < c ? x[p * c + ch] : 0.f);
  }
}

// FP32 [P][16] -> FP32 [P][c]
__global__ __launch_bounds__(256) void k_from16(long P, int c, const float* __restrict__ y16,
                                                float* __restrict__ y) {
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < P * c; e += (long)gridDim.x * 256)
    y[e] = y16[(e / c) * kCP + e % c];
}

// FP32 [P][c] -> BF16 [P][16] gradient seed
__global__ __launch_bounds__(256) void k_dy_to_bf(long P, int c, const float* __restrict__ dy,
                                                  uint16_t* __restrict__ d) {
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < P * kCP; e += (long)gridDim.x * 256) {
    const int ch = int(e % kCP);
    d[e] = f2bf(ch < c ? dy[(e / kCP) * c + ch] : 0.f);
  }
}

// per-sample partial sums of ||y - e||^2 and ||e||^2 (grid: (blocks, batch))
__global__ __launch_bounds__(256) void k_loss_part(long Pb, int c, const float* __restrict__ y16,
                                                   const float* __restrict__ e,
                                                   double* __restrict__ num,
                                                   double* __restrict__ den) {
  const int s = blockIdx.y;
  double a = 0.0, b = 0.0;
  for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < Pb * c; q += (long)gridDim.x * 256) {
    const long p = q / c;
    const int ch = int(q % c);
    const double ev = e[(size_t)s * Pb * c + q];
    const double d = double(y16[((size_t)s * Pb + p) * kCP + ch]) - ev;
    a += d * d;
    b += ev * ev;
  }
  __shared__ double sh[4];
  double t = block_sum<256>(a, sh);
  if (threadIdx.x == 0) num[s * gridDim.x + blockIdx.x] = t;
  __syncthreads();
  t = block_sum<256>(b, sh);
  if (threadIdx.x == 0) den[s * gridDim.x + blockIdx.x] = t;
}

// mean squared error over all batch entries (scalar[0]) and the per-sample
// weight 1 / (points * channels) (scalar[1 + s]) from the partials (one
// block of 256 threads, fixed order); inputs and targets are already
// normalised by the residual scale
__global__ __launch_bounds__(256) void k_loss_final(int batch, int nblk, long per_sample,
                                                    const double* num, double* scal) {
  __shared__ double sh[4];
  double L = 0.0;
  const double inv = 1.0 / double(per_sample);
  for (int s = 0; s < batch; ++s) {
    double a = 0.0;
    for (int k = threadIdx.x; k < nblk; k += 256) a += num[s * nblk + k];
    a = block_sum<256>(a, sh);  // valid in thread 0
    __syncthreads();            // sh is reused by the next sample
    if (threadIdx.x == 0) {
      scal[1 + s] = inv;
      L += a * inv;
    }
  }
  if (threadIdx.x == 0) scal[0] = L / batch;
}

// dz = 2 (y - e) / (points * channels * batch), BF16 [P][16]
__global__ __launch_bounds__(256) void k_loss_grad(long Pb, int c, int batch,
                                                   const float* __restrict__ y16,
                                                   const float* __restrict__ e,
                                                   const double* __restrict__ scal,
                                                   uint16_t* __restrict__ dz) {
  const long P = Pb * batch;
  for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < P * kCP; q += (long)gridDim.x * 256) {
    const long p = q / kCP;
    const int ch = int(q % kCP);
    float v = 0.f;
    if (ch < c) {
      const int s = int(p / Pb);
      const double ev = e[p * c + ch];
      v = float(2.0 * (double(y16[q]) - ev) * scal[1 + s] / batch);
    }
    dz[q] = f2bf(v);
  }
}

__global__ __launch_bounds__(256) void k_adam(int n, float* __restrict__ w,
                                              const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    w[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// gather crops: inputs [pairs][P][cin] -> act BF16 [B][crop^d][16],
// targets [pairs][P][cout] -> e FP32 [B][crop^d][cout]; desc[s] = {pair, ox, oy, oz}
__global__ __launch_bounds__(256) void k_gather(int nx, int ny, int nz, int dim, int crop, int cin,
                                                int cout, const float* __restrict__ inputs,
                                                const float* __restrict__ targets,
                                                const int* __restrict__ desc,
                                                uint16_t* __restrict__ act, float* __restrict__ e) {
  const int s = blockIdx.y;
  const int cz = dim == 3 ? crop : 1;
  const long Pc = (long)crop * crop * cz;
  const long P = (long)nx * ny * nz;
  const int pair = desc[4 * s], ox = desc[4 * s + 1], oy = desc[4 * s + 2], oz = desc[4 * s + 3];
  for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < Pc; q += (long)gridDim.x * 256) {
    const int i = int(q % crop), j = int((q / crop) % crop), k = int(q / ((long)crop * crop));
    const long src = ((long)(k + oz) * ny + (j + oy)) * nx + (i + ox);
    const float* xi = inputs + ((size_t)pair * P + src) * cin;
    uint16_t* a = act + ((size_t)s * Pc + q) * kCP;
    for (int ch = 0; ch < kCP; ++ch) a[ch] = f2bf(ch < cin ? xi[ch] : 0.f);
    const float* ti = targets + ((size_t)pair * P + src) * cout;
    float* eo = e + ((size_t)s * Pc + q) * cout;
    for (int ch = 0; ch < cout; ++ch) eo[ch] = ti[ch];
  }
}

}  // namespace gkb

// --------------------------------------------------------------- network

struct gkb_cnn {
  int dim = 3, L = 0, taps = 27;
  int ch[gkb::kMaxLayers + 1] = {0};
  long np = 0;
  long off[gkb::kMaxLayers + 1] = {0};  // flat offset of each layer
  float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *wf = nullptr, *wd = nullptr;  // [L][taps][256]
  float* bias = nullptr;                  // [L][16]
  int adam_t = 0;
  // workspace (grown on demand)
  long cap = 0;
  uint16_t* act[gkb::kMaxLayers] = {nullptr};
  uint16_t *dz0 = nullptr, *dz1 = nullptr;
  float* y16 = nullptr;
  float* pad = nullptr;    // padded grad of one layer
  float* wpart = nullptr;  // wgrad block partials
  int wblk = 0;
  double* lscal = nullptr;  // loss scalars
  double *lnum = nullptr, *lden = nullptr;
  int lcap = 0;
  float* ebuf = nullptr;  // training targets
  long ecap = 0;
  int* desc = nullptr;
  int dcap = 0;
  hipStream_t s = nullptr;
  bool weights_dirty = true;
};

namespace {

#define CNNCK(expr)                                                              \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      std::fprintf(stderr, "gkb_cnn: HIP error %s at %s:%d\n", hipGetErrorString(e_), \
                   __FILE__, __LINE__);                                          \
      return GKB_EHIP;                                                           \
    }                                                                            \
  } while (0)

// Host <-> device copy ordered on the network's (non-blocking) stream and
// complete on return
hipError_t cnn_copy(gkb_cnn* n, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, n->s);
  return e != hipSuccess ? e : hipStreamSynchronize(n->s);
}

int cnn_grid(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 8192)); }

int cnn_prepare_weights(gkb_cnn* n) {
  if (!n->weights_dirty) return GKB_OK;
  for (int l = 0; l < n->L; ++l)
    gkb::k_pack_weights<<<cnn_grid(n->taps * 256), 256, 0, n->s>>>(
        n->params + n->off[l], n->taps, n->ch[l], n->ch[l + 1], n->wf + (size_t)l * n->taps * 256,
        n->wd + (size_t)l * n->taps * 256, n->bias + 16 * l);
  CNNCK(hipGetLastError());
  n->weights_dirty = false;
  return GKB_OK;
}

int cnn_reserve(gkb_cnn* n, long P) {
  // point indices are decomposed in 32-bit arithmetic (coords)
  if (P <= 0 || P > 0x7fffffffL) return GKB_EINVAL;
  if (P <= n->cap) return GKB_OK;
  for (int l = 0; l < n->L; ++l) {
    if (n->act[l]) (void)hipFree(n->act[l]);
    CNNCK(hipMalloc(&n->act[l], P * gkb::kCP * sizeof(uint16_t)));
  }
  if (n->dz0) (void)hipFree(n->dz0);
  if (n->dz1) (void)hipFree(n->dz1);
  if (n->y16) (void)hipFree(n->y16);
  CNNCK(hipMalloc(&n->dz0, P * gkb::kCP * sizeof(uint16_t)));
  CNNCK(hipMalloc(&n->dz1, P * gkb::kCP * sizeof(uint16_t)));
  CNNCK(hipMalloc(&n->y16, P * gkb::kCP * sizeof(float)));
  n->cap = P;
  return GKB_OK;
}

template <int DIM>
void cnn_forward_dim(gkb_cnn* n, const gkb::CnnGeom& g) {
  const int blocks = gkb::conv_blocks(g.P);
  for (int l = 0; l < n->L; ++l) {
    const uint16_t* w = n->wf + (size_t)l * n->taps * 256;
    const float* b = n->bias + 16 * l;
    if (l < n->L - 1)
      gkb::launch_conv<DIM, gkb::kOutReluBf16>(n->ch[l], blocks, n->s, g, n->act[l], w, b,
                                               n->act[l + 1], nullptr);
    else
      gkb::launch_conv<DIM, gkb::kOutF32>(n->ch[l], blocks, n->s, g, n->act[l], w, b, n->y16,
                                          nullptr);
  }
}

// forward from n->act[0] (already filled) into n->y16
int cnn_forward_act(gkb_cnn* n, const gkb::CnnGeom& g) {
  int rc = cnn_prepare_weights(n);
  if (rc) return rc;
  if (n->dim == 2) cnn_forward_dim<2>(n, g);
  else cnn_forward_dim<3>(n, g);
  CNNCK(hipGetLastError());
  return GKB_OK;
}

template <int DIM>
int cnn_backward_dim(gkb_cnn* n, const gkb::CnnGeom& g, float* dx16) {
  constexpr int TAPS = DIM == 2 ? 9 : 27;
  const int NP = TAPS * 256 + 16;
  const int wblk = (int)std::max<long>(1, std::min<long>((g.P + 1023) / 1024, 512));
  if (wblk > n->wblk) {
    if (n->wpart) (void)hipFree(n->wpart);
    CNNCK(hipMalloc(&n->wpart, (size_t)wblk * NP * sizeof(float)));
    n->wblk = wblk;
  }
  const int blocks = gkb::conv_blocks(g.P);
  uint16_t* dz = n->dz0;
  uint16_t* dzn = n->dz1;
  for (int l = n->L - 1; l >= 0; --l) {
    if (n->ch[l] <= 4)
      gkb::k_wgrad<DIM, 4><<<wblk, 256, 0, n->s>>>(g, n->act[l], dz, n->wpart);
    else if (n->ch[l] <= 8)
      gkb::k_wgrad<DIM, 8><<<wblk, 256, 0, n->s>>>(g, n->act[l], dz, n->wpart);
    else
      gkb::k_wgrad<DIM, 16><<<wblk, 256, 0, n->s>>>(g, n->act[l], dz, n->wpart);
    gkb::k_wgrad_reduce<<<(NP + gkb::kRedOut - 1) / gkb::kRedOut, 256, 0, n->s>>>(n->wpart, wblk,
                                                                                 NP, n->pad);
    gkb::k_grad_flat<<<cnn_grid(TAPS * 256 + 16), 256, 0, n->s>>>(n->pad, TAPS, n->ch[l],
                                                                   n->ch[l + 1], n->grad + n->off[l]);
    const uint16_t* wd = n->wd + (size_t)l * TAPS * 256;
    // the adjoint convolution reads the layer's output channels
    if (l > 0) {
      gkb::launch_conv<DIM, gkb::kOutMaskBf16>(n->ch[l + 1], blocks, n->s, g, dz, wd, nullptr,
                                               dzn, n->act[l]);
      std::swap(dz, dzn);
    } else if (dx16) {
      gkb::launch_conv<DIM, gkb::kOutF32>(n->ch[l + 1], blocks, n->s, g, dz, wd, nullptr, dx16,
                                          nullptr);
    }
  }
  CNNCK(hipGetLastError());
  return GKB_OK;
}

int cnn_backward_act(gkb_cnn* n, const gkb::CnnGeom& g, float* dx16) {
  int rc = cnn_prepare_weights(n);
  if (rc) return rc;
  return n->dim == 2 ? cnn_backward_dim<2>(n, g, dx16) : cnn_backward_dim<3>(n, g, dx16);
}

int cnn_adam(gkb_cnn* n, double lr, double b1, double b2, double eps) {
  n->adam_t += 1;
  const float c1 = float(1.0 - std::pow(b1, n->adam_t)), c2 = float(1.0 - std::pow(b2, n->adam_t));
  gkb::k_adam<<<cnn_grid(n->np), 256, 0, n->s>>>((int)n->np, n->params, n->grad, n->m, n->v,
                                                  float(lr), float(b1), float(b2), float(eps), c1,
                                                  c2);
  n->weights_dirty = true;
  CNNCK(hipGetLastError());
  return GKB_OK;
}

int cnn_loss_buffers(gkb_cnn* n, int batch, int nblk) {
  if (batch * nblk > n->lcap) {
    if (n->lnum) (void)hipFree(n->lnum);
    if (n->lden) (void)hipFree(n->lden);
    CNNCK(hipMalloc(&n->lnum, (size_t)batch * nblk * sizeof(double)));
    CNNCK(hipMalloc(&n->lden, (size_t)batch * nblk * sizeof(double)));
    n->lcap = batch * nblk;
  }
  if (!n->lscal) CNNCK(hipMalloc(&n->lscal, 1025 * sizeof(double)));
  return GKB_OK;
}

}  // namespace

extern "C" {

int gkb_cnn_create(int dim, int n_layers, const int* channels, unsigned seed, gkb_cnn** out) {
  if (!out || !channels || (dim != 2 && dim != 3) || n_layers < 1 || n_layers > gkb::kMaxLayers)
    return GKB_EINVAL;
  for (int l = 0; l <= n_layers; ++l)
    if (channels[l] < 1 || channels[l] > gkb::kCP) return GKB_EINVAL;
  gkb_cnn* n = new gkb_cnn();
  n->dim = dim;
  n->L = n_layers;
  n->taps = dim == 2 ? 9 : 27;
  long o = 0;
  for (int l = 0; l <= n_layers; ++l) n->ch[l] = channels[l];
  for (int l = 0; l < n_layers; ++l) {
    n->off[l] = o;
    o += (long)n->taps * channels[l] * channels[l + 1] + channels[l + 1];
  }
  n->np = o;
  auto fail = [&](int rc) {
    gkb_cnn_destroy(n);
    return rc;
  };
  if (hipStreamCreateWithFlags(&n->s, hipStreamNonBlocking) != hipSuccess) return fail(GKB_EHIP);
  float** fp[] = {&n->params, &n->grad, &n->m, &n->v};
  for (auto p : fp) {
    if (hipMalloc(p, n->np * sizeof(float)) != hipSuccess) return fail(GKB_ENOMEM);
    if (hipMemsetAsync(*p, 0, n->np * sizeof(float), n->s) != hipSuccess) return fail(GKB_EHIP);
  }
  if (hipMalloc(&n->wf, (size_t)n_layers * n->taps * 256 * 2) != hipSuccess ||
      hipMalloc(&n->wd, (size_t)n_layers * n->taps * 256 * 2) != hipSuccess ||
      hipMalloc(&n->bias, (size_t)n_layers * 16 * 4) != hipSuccess ||
      hipMalloc(&n->pad, (size_t)(27 * 256 + 16) * 4) != hipSuccess)
    return fail(GKB_ENOMEM);
  // seeded He-uniform initialisation (64-bit LCG), zero biases
  std::vector<float> h(n->np, 0.f);
  uint64_t st = 0x9E3779B97F4A7C15ull ^ seed;
  for (int l = 0; l < n_layers; ++l) {
    const int fan_in = n->taps * channels[l];
    const float lim = std::sqrt(6.0f / fan_in);
    const long nw = (long)n->taps * channels[l] * channels[l + 1];
    for (long e = 0; e < nw; ++e) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      const double u = double(st >> 11) * (1.0 / 9007199254740992.0);
      h[n->off[l] + e] = float((2.0 * u - 1.0) * lim);
    }
  }
  if (cnn_copy(n, n->params, h.data(), n->np * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail(GKB_EHIP);
  *out = n;
  return GKB_OK;
}

void gkb_cnn_destroy(gkb_cnn* n) {
  if (!n) return;
  if (n->s) (void)hipStreamSynchronize(n->s);
  void* ptrs[] = {n->params, n->grad, n->m,    n->v,    n->wf,    n->wd,   n->bias,
                  n->dz0,    n->dz1,  n->y16,  n->pad,  n->wpart, n->lscal, n->lnum,
                  n->lden,   n->ebuf, n->desc};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int l = 0; l < gkb::kMaxLayers; ++l)
    if (n->act[l]) (void)hipFree(n->act[l]);
  if (n->s) (void)hipStreamDestroy(n->s);
  delete n;
}

long gkb_cnn_param_count(const gkb_cnn* n) { return n ? n->np : -1; }

int gkb_cnn_set_params(gkb_cnn* n, const float* hp) {
  if (!n || !hp) return GKB_EINVAL;
  CNNCK(cnn_copy(n, n->params, hp, n->np * 4, hipMemcpyHostToDevice));
  n->weights_dirty = true;
  return GKB_OK;
}

int gkb_cnn_get_params(const gkb_cnn* n, float* hp) {
  if (!n || !hp) return GKB_EINVAL;
  CNNCK(cnn_copy(const_cast<gkb_cnn*>(n), hp, n->params, n->np * 4, hipMemcpyDeviceToHost));
  return GKB_OK;
}

int gkb_cnn_forward(gkb_cnn* n, int nx, int ny, int nz, int batch, const float* x, float* y) {
  // inputs may come from any stream: wait for all submitted device work
  CNNCK(hipDeviceSynchronize());
  if (!n || !x || !y || nx < 1 || ny < 1 || nz < 1 || batch < 1 || (n->dim == 2 && nz != 1))
    return GKB_EINVAL;
  gkb::CnnGeom g{nx, ny, nz, batch, (long)nx * ny * nz * batch};
  int rc = cnn_reserve(n, g.P);
  if (rc) return rc;
  gkb::k_to_act<<<cnn_grid(g.P * 16), 256, 0, n->s>>>(g.P, n->ch[0], x, n->act[0]);
  rc = cnn_forward_act(n, g);
  if (rc) return rc;
  gkb::k_from16<<<cnn_grid(g.P * n->ch[n->L]), 256, 0, n->s>>>(g.P, n->ch[n->L], n->y16, y);
  CNNCK(hipStreamSynchronize(n->s));
  return GKB_OK;
}

int gkb_cnn_backward(gkb_cnn* n, int nx, int ny, int nz, int batch, const float* x,
                     const float* dy, float* dx, float* grad_host) {
  // inputs may come from any stream: wait for all submitted device work
  CNNCK(hipDeviceSynchronize());
  if (!n || !x || !dy || nx < 1 || ny < 1 || nz < 1 || batch < 1 || (n->dim == 2 && nz != 1))
    return GKB_EINVAL;
  gkb::CnnGeom g{nx, ny, nz, batch, (long)nx * ny * nz * batch};
  int rc = cnn_reserve(n, g.P);
  if (rc) return rc;
  gkb::k_to_act<<<cnn_grid(g.P * 16), 256, 0, n->s>>>(g.P, n->ch[0], x, n->act[0]);
  rc = cnn_forward_act(n, g);
  if (rc) return rc;
  gkb::k_dy_to_bf<<<cnn_grid(g.P * 16), 256, 0, n->s>>>(g.P, n->ch[n->L], dy, n->dz0);
  float* dx16 = nullptr;
  if (dx) dx16 = n->y16;  // the forward output is no longer needed
  rc = cnn_backward_act(n, g, dx16);
  if (rc) return rc;
  if (dx) gkb::k_from16<<<cnn_grid(g.P * n->ch[0]), 256, 0, n->s>>>(g.P, n->ch[0], dx16, dx);
  if (grad_host) CNNCK(hipMemcpyAsync(grad_host, n->grad, n->np * 4, hipMemcpyDeviceToHost, n->s));
  CNNCK(hipStreamSynchronize(n->s));
  return GKB_OK;
}

int gkb_cnn_adam_step(gkb_cnn* n, const float* grad_host, double lr, double b1, double b2,
                      double eps) {
  if (!n) return GKB_EINVAL;
  if (grad_host) CNNCK(cnn_copy(n, n->grad, grad_host, n->np * 4, hipMemcpyHostToDevice));
  int rc = cnn_adam(n, lr, b1, b2, eps);
  if (rc) return rc;
  CNNCK(hipStreamSynchronize(n->s));
  return GKB_OK;
}

int gkb_cnn_train(gkb_cnn* n, const float* inputs, const float* targets, int n_pairs, int nx,
                  int ny, int nz, int crop, int batch, int steps, double lr, unsigned seed,
                  float* loss_host) {
  // inputs may come from any stream: wait for all submitted device work
  CNNCK(hipDeviceSynchronize());
  if (!n || !inputs || !targets || n_pairs < 1 || batch < 1 || batch > 1024 || steps < 0 ||
      crop < 3 || crop > nx || crop > ny || (n->dim == 3 && crop > nz) || (n->dim == 2 && nz != 1))
    return GKB_EINVAL;
  const int dim = n->dim, cin = n->ch[0], cout = n->ch[n->L];
  const long Pc = (long)crop * crop * (dim == 3 ? crop : 1);
  gkb::CnnGeom g{crop, crop, dim == 3 ? crop : 1, batch, Pc * batch};
  int rc = cnn_reserve(n, g.P);
  if (rc) return rc;
  if (g.P * cout > n->ecap) {
    if (n->ebuf) (void)hipFree(n->ebuf);
    CNNCK(hipMalloc(&n->ebuf, g.P * cout * sizeof(float)));
    n->ecap = g.P * cout;
  }
  if (batch > n->dcap) {
    if (n->desc) (void)hipFree(n->desc);
    CNNCK(hipMalloc(&n->desc, batch * 4 * sizeof(int)));
    n->dcap = batch;
  }
  const int lblk = (int)std::max<long>(1, std::min<long>((Pc * cout + 255) / 256, 256));
  rc = cnn_loss_buffers(n, batch, lblk);
  if (rc) return rc;
  std::vector<int> desc(4 * batch);
  uint64_t st = 0xD1B54A32D192ED03ull ^ ((uint64_t)seed << 1);
  auto rnd = [&](int mod) {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return int((st >> 33) % (uint64_t)mod);
  };
  double hl[1];
  for (int it = 0; it < steps; ++it) {
    for (int s = 0; s < batch; ++s) {
      desc[4 * s] = rnd(n_pairs);
      desc[4 * s + 1] = rnd(nx - crop + 1);
      desc[4 * s + 2] = rnd(ny - crop + 1);
      desc[4 * s + 3] = dim == 3 ? rnd(nz - crop + 1) : 0;
    }
    CNNCK(hipMemcpyAsync(n->desc, desc.data(), 4 * batch * sizeof(int), hipMemcpyHostToDevice, n->s));
    gkb::k_gather<<<dim3(cnn_grid(Pc), batch), 256, 0, n->s>>>(
        nx, ny, nz, dim, crop, cin, cout, inputs, targets, n->desc, n->act[0], n->ebuf);
    rc = cnn_forward_act(n, g);
    if (rc) return rc;
    gkb::k_loss_part<<<dim3(lblk, batch), 256, 0, n->s>>>(Pc, cout, n->y16, n->ebuf, n->lnum,
                                                          n->lden);
    gkb::k_loss_final<<<1, 256, 0, n->s>>>(batch, lblk, Pc * cout, n->lnum, n->lscal);
    gkb::k_loss_grad<<<cnn_grid(g.P * 16), 256, 0, n->s>>>(Pc, cout, batch, n->y16, n->ebuf,
                                                           n->lscal, n->dz0);
    rc = cnn_backward_act(n, g, nullptr);
    if (rc) return rc;
    rc = cnn_adam(n, lr, 0.9, 0.999, 1e-8);
    if (rc) return rc;
    if (loss_host) {
      CNNCK(hipMemcpyAsync(hl, n->lscal, sizeof(double), hipMemcpyDeviceToHost, n->s));
      CNNCK(hipStreamSynchronize(n->s));
      loss_host[it] = float(hl[0]);
    }
  }
  CNNCK(hipStreamSynchronize(n->s));
  return GKB_OK;
}

int gkb_cnn_eval(gkb_cnn* n, const float* inputs, const float* targets, int n_pairs, int nx,
                 int ny, int nz, double* loss) {
  // inputs may come from any stream: wait for all submitted device work
  CNNCK(hipDeviceSynchronize());
  if (!n || !inputs || !targets || !loss || n_pairs < 1 || (n->dim == 2 && nz != 1))
    return GKB_EINVAL;
  const int cin = n->ch[0], cout = n->ch[n->L];
  const long P = (long)nx * ny * nz;
  gkb::CnnGeom g{nx, ny, nz, 1, P};
  int rc = cnn_reserve(n, P);
  if (rc) return rc;
  const int lblk = (int)std::max<long>(1, std::min<long>((P * cout + 255) / 256, 256));
  rc = cnn_loss_buffers(n, 1, lblk);
  if (rc) return rc;
  double total = 0.0, hl[1];
  for (int k = 0; k < n_pairs; ++k) {
    gkb::k_to_act<<<cnn_grid(P * 16), 256, 0, n->s>>>(P, cin, inputs + (size_t)k * P * cin,
                                                      n->act[0]);
    rc = cnn_forward_act(n, g);
    if (rc) return rc;
    gkb::k_loss_part<<<dim3(lblk, 1), 256, 0, n->s>>>(P, cout, n->y16,
                                                      targets + (size_t)k * P * cout, n->lnum,
                                                      n->lden);
    gkb::k_loss_final<<<1, 256, 0, n->s>>>(1, lblk, P * cout, n->lnum, n->lscal);
    CNNCK(hipMemcpyAsync(hl, n->lscal, sizeof(double), hipMemcpyDeviceToHost, n->s));
    CNNCK(hipStreamSynchronize(n->s));
    total += hl[0];
  }
  *loss = total / n_pairs;
  return GKB_OK;
}

int gkb_cnn_save(const gkb_cnn* n, const char* path) {
  if (!n || !path) return GKB_EINVAL;
  std::vector<float> p(n->np), m(n->np), v(n->np);
  gkb_cnn* nn = const_cast<gkb_cnn*>(n);
  CNNCK(cnn_copy(nn, p.data(), n->params, n->np * 4, hipMemcpyDeviceToHost));
  CNNCK(cnn_copy(nn, m.data(), n->m, n->np * 4, hipMemcpyDeviceToHost));
  CNNCK(cnn_copy(nn, v.data(), n->v, n->np * 4, hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) return GKB_EINVAL;
  const char magic[8] = {'G', 'K', 'B', 'C', 'N', 'N', '0', '1'};
  int hdr[4 + gkb::kMaxLayers + 1] = {1, n->dim, n->L, n->adam_t};
  for (int l = 0; l <= n->L; ++l) hdr[4 + l] = n->ch[l];
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
            std::fwrite(p.data(), 4, n->np, f) == (size_t)n->np &&
            std::fwrite(m.data(), 4, n->np, f) == (size_t)n->np &&
            std::fwrite(v.data(), 4, n->np, f) == (size_t)n->np;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? GKB_OK : GKB_EINVAL;
}

int gkb_cnn_load(const char* path, gkb_cnn** out) {
  if (!path || !out) return GKB_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return GKB_EINVAL;
  char magic[8];
  int hdr[4 + gkb::kMaxLayers + 1];
  if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "GKBCNN01", 8) != 0 ||
      std::fread(hdr, sizeof(hdr), 1, f) != 1 || hdr[0] != 1 || hdr[2] < 1 ||
      hdr[2] > gkb::kMaxLayers) {
    std::fclose(f);
    return GKB_EINVAL;
  }
  gkb_cnn* n = nullptr;
  int rc = gkb_cnn_create(hdr[1], hdr[2], hdr + 4, 0, &n);
  if (rc) {
    std::fclose(f);
    return rc;
  }
  std::vector<float> p(n->np), m(n->np), v(n->np);
  bool ok = std::fread(p.data(), 4, n->np, f) == (size_t)n->np &&
            std::fread(m.data(), 4, n->np, f) == (size_t)n->np &&
            std::fread(v.data(), 4, n->np, f) == (size_t)n->np;
  std::fclose(f);
  if (!ok) {
    gkb_cnn_destroy(n);
    return GKB_EINVAL;
  }
  n->adam_t = hdr[3];
  if (cnn_copy(n, n->params, p.data(), n->np * 4, hipMemcpyHostToDevice) != hipSuccess ||
      cnn_copy(n, n->m, m.data(), n->np * 4, hipMemcpyHostToDevice) != hipSuccess ||
      cnn_copy(n, n->v, v.data(), n->np * 4, hipMemcpyHostToDevice) != hipSuccess) {
    gkb_cnn_destroy(n);
    return GKB_EHIP;
  }
  *out = n;
  return GKB_OK;
}

}  // extern "C"
