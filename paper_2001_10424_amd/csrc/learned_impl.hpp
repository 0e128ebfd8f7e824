// Learned inner solve (included by gkb.hip after the context type):
// flexible CG (FCG(1), Polak-Ribiere beta) on M x = f with the preconditioner
//     z = V(r) + theta c,  c = (s / lambda) unpack(C_theta(pack(rt) / s)),
//     rt = r - M V(r) (the residual the V-cycle leaves), s = RMS(rt),
//     lambda = mean diag(W), theta = (c . rt) / (c . M c) (energy-optimal step)
// and plain multigrid-PCG as the fallback, plus capture of training pairs
// from multigrid-PCG inner solves.
#pragma once

struct Learned {
  gkb_cnn* net = nullptr;
  // once the network direction has failed a guard, the rest of the
  // gkb_solve uses MG-PCG
  bool off = false;
  // network energy gain relative to the V-cycle over the current gkb_solve
  double gain_sum = 0.0;
  long gain_n = 0;
  double lam = 1.0;       // mean diag(W) over the unknown faces
  long m_unknown = 1;
  float* logmu = nullptr;  // cell log-viscosity (input channel), zeros for mu = 1
  // FCG work vectors (inner precision stored as raw bytes)
  void* zv = nullptr;
  // capture
  float* cap_in = nullptr;
  float* cap_tg = nullptr;
  int cap_max = 0, cap_n = 0;
  std::vector<int> cap_iters;
  std::vector<void*> snaps;  // 2 * n_iters vectors (r_i, x_i) in inner precision
  void* tmp = nullptr;
};

namespace gkb {

// squared norm of the post-V-cycle residual from block partials
__global__ __launch_bounds__(kFinal) void k_set_rt2(PcgState* st, const double* part, int n) {
  if (st->done || st->fallback) return;
  __shared__ double sh[kFinal / 64];
  const double v = sum_partials(part, n, sh);
  if (threadIdx.x == 0) st->rt2 = v;
}

// cell-packed input channels: the post-V-cycle residual of the faces below /
// left of the cell scaled by 1/s (s = sqrt(rt.rt / m_unknown)), then log(mu)
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_pack_faces(Grid G, const T* __restrict__ r,
                                                    const PcgState* __restrict__ st, double mu_n,
                                                    const float* __restrict__ logmu,
                                                    uint16_t* __restrict__ act) {
  if (st->done || st->fallback) return;
  const double s = sqrt(st->rt2 / mu_n);
  const float inv = s > 0.0 ? float(1.0 / s) : 0.f;
  const long nc = G.n_cells;
  for (long c = (long)blockIdx.x * 256 + threadIdx.x; c < nc; c += (long)gridDim.x * 256) {
    const int i = int(c % G.n[0]), j = int((c / G.n[0]) % G.n[1]), k = int(c / ((long)G.n[0] * G.n[1]));
    uint16_t* a = act + c * kCP;
    a[0] = f2bf(float(r[fidx<0>(G, i, j, k)]) * inv);
    a[1] = f2bf(float(r[fidx<1>(G, i, j, k)]) * inv);
    int ch = 2;
    if (DIM == 3) a[ch++] = f2bf(float(r[fidx<2>(G, i, j, k)]) * inv);
    a[ch++] = f2bf(logmu[c]);
    for (; ch < kCP; ++ch) a[ch] = 0;
  }
}

// correction c = (s / lambda) y16[cell][component] on unknown faces that are
// the lower face of a cell, 0 elsewhere; partial c.rt
template <typename T, int DIM, int C>
__device__ __forceinline__ void unpack_face(const Grid& G, int idx, int k,
                                            const float* __restrict__ y16, float scale,
                                            const T* __restrict__ rt, T* __restrict__ cv,
                                            double& a) {
  const int e0 = G.ext[C][0], e1 = G.ext[C][1];
  if (idx >= e0 * e1 || k >= G.ext[C][2]) return;
  const int j = idx / e0, i = idx - j * e0;
  const int f = fidx<C>(G, i, j, k);
  const int ic = C == 0 ? i : (C == 1 ? j : k);
  T v = T(0);
  if (unk<C>(G, ic) && ic < G.n[C]) v = T(scale * y16[(long)cidx(G, i, j, k) * kCP + C]);
  cv[f] = v;
  a += double(v) * double(rt[f]);
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_unpack_c(Grid G, const float* __restrict__ y16,
                                                  const PcgState* __restrict__ st, double mu_n,
                                                  double lam, const T* __restrict__ rt,
                                                  T* __restrict__ cv, double* __restrict__ p_crt) {
  if (st->done || st->fallback) return;
  const float scale = float(sqrt(st->rt2 / mu_n) / lam);
  const int c = blockIdx.z / G.nze, k = blockIdx.z - c * G.nze;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  double a = 0.0;
  if (c == 0) unpack_face<T, DIM, 0>(G, idx, k, y16, scale, rt, cv, a);
  else if (c == 1) unpack_face<T, DIM, 1>(G, idx, k, y16, scale, rt, cv, a);
  else if (DIM == 3) unpack_face<T, DIM, 2>(G, idx, k, y16, scale, rt, cv, a);
  __shared__ double sh[4];
  double t = block_sum<256>(a, sh);
  if (threadIdx.x == 0) p_crt[blockIdx.z * gridDim.x + blockIdx.x] = t;
}

// theta = (c . rt) / (c . M c): the step along c that minimises the energy
// norm of the error left by the V-cycle, M^-1 rt - theta c
__global__ __launch_bounds__(kFinal) void k_set_theta(PcgState* st, const double* p_crt, int n1,
                                                      const double* p_cmc, int n2) {
  if (st->done || st->fallback) return;
  __shared__ double sh[kFinal / 64];
  const double crt = sum_partials(p_crt, n1, sh);
  __syncthreads();
  const double cmc = sum_partials(p_cmc, n2, sh);
  if (threadIdx.x == 0) {
    const bool ok = cmc > 0.0 && isfinite(crt / cmc);
    st->theta = ok ? crt / cmc : 0.0;
    st->gain = ok ? crt * crt / cmc : 0.0;
  }
}

// z = zv + theta c (z = zv during fallback); partials r.z, z.r_prev, zv.r_prev
template <typename T>
__global__ __launch_bounds__(256) void k_combine(int n, const PcgState* __restrict__ st,
                                                 const T* __restrict__ zv, const T* __restrict__ cv,
                                                 const T* __restrict__ r, const T* __restrict__ rp,
                                                 T* __restrict__ z, double* __restrict__ p_rz,
                                                 double* __restrict__ p_zrp,
                                                 double* __restrict__ p_zvrp) {
  if (st->done) return;
  const T th = st->fallback ? T(0) : T(st->theta);
  double a = 0.0, b = 0.0, c2 = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const T zvi = zv[i];
    const T v = zvi + th * cv[i];
    z[i] = v;
    const double rpi = double(rp[i]);
    a += double(r[i]) * double(v);
    b += double(v) * rpi;
    c2 += double(zvi) * rpi;
  }
  __shared__ double sh[4];
  double t = block_sum<256>(a, sh);
  if (threadIdx.x == 0) p_rz[blockIdx.x] = t;
  __syncthreads();
  t = block_sum<256>(b, sh);
  if (threadIdx.x == 0) p_zrp[blockIdx.x] = t;
  __syncthreads();
  t = block_sum<256>(c2, sh);
  if (threadIdx.x == 0) p_zvrp[blockIdx.x] = t;
}

// r_prev = r; x += alpha p; r -= alpha q; partial r.r
template <typename T>
__global__ __launch_bounds__(256) void k_fcg_xr(int n, const PcgState* __restrict__ st,
                                                const T* __restrict__ p, const T* __restrict__ q,
                                                T* __restrict__ x, T* __restrict__ r,
                                                T* __restrict__ rp, double* __restrict__ part_rr) {
  if (st->done) return;
  const T a = T(st->alpha);
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const T ri = r[i];
    rp[i] = ri;
    x[i] += a * p[i];
    const T rn = ri - a * q[i];
    r[i] = rn;
    s += double(rn) * double(rn);
  }
  __shared__ double sh[4];
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
}

// choose the direction: the CNN-corrected z unless it fails the descent test
// (r.z <= 0), the residual stagnated (no decrease over 50 iterations) or the
// network step removes less than min_gain of the V-cycle step's error energy
// (the option learned_min_gain: one application costs about as much as a
// V-cycle, so a much smaller gain cannot pay for itself; min_gain = 0 turns
// this test off, min_gain < 0 the progress test too, leaving only the
// descent test that flexible CG needs); then fall back to the V-cycle alone
// for the rest of the solve, restarting CG.  first = 1 at the start of a
// solve.
__global__ __launch_bounds__(kFinal) void k_fcg_beta(PcgState* st, const double* p_rzv, int nv,
                                                     const double* p_rz, const double* p_zrp,
                                                     const double* p_zvrp, int nu, int first,
                                                     double min_gain) {
  if (st->done) return;
  __shared__ double sh[kFinal / 64];
  const double rzv = sum_partials(p_rzv, nv, sh);
  __syncthreads();
  const double rz = sum_partials(p_rz, nu, sh);
  __syncthreads();
  const double zrp = sum_partials(p_zrp, nu, sh);
  __syncthreads();
  const double zvrp = sum_partials(p_zvrp, nu, sh);
  if (threadIdx.x != 0) return;
  bool restart = first != 0;
  if (!st->fallback) {
    const double ratio = rzv > 0.0 ? st->gain / rzv : 0.0;
    st->gain_sum += ratio;
    st->gain_n += 1;
    const bool low = min_gain > 0.0 && ratio < min_gain;
    const bool stalled = min_gain >= 0.0 && st->stagnant;
    const int reason = !(rz > 0.0) ? 1 : (stalled ? 2 : (low ? 3 : 0));
    if (reason) {
      st->fallback = 1;
      st->fallbacks += 1;
      st->fb_it = st->it;
      st->fb_reason = reason;
      restart = true;
    }
  }
  st->use_zv = st->fallback;
  const double rz_use = st->fallback ? rzv : rz;
  const double zr_use = st->fallback ? zvrp : zrp;
  st->beta = restart ? 0.0 : (rz_use - zr_use) / st->rz;
  st->rz = rz_use;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fcg_p(int n, const PcgState* __restrict__ st,
                                               const T* __restrict__ z, const T* __restrict__ zv,
                                               T* __restrict__ p) {
  if (st->done) return;
  const T b = T(st->beta);
  const T* src = st->use_zv ? zv : z;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = src[i] + b * p[i];
}

// training pair of one snapshot: input [cells][dim+1], target [cells][dim]
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_pack_pair(Grid G, const T* __restrict__ r,
                                                   const T* __restrict__ et, double inv_s,
                                                   double lam_over_s, const float* __restrict__ logmu,
                                                   float* __restrict__ in, float* __restrict__ tg) {
  const long nc = G.n_cells;
  for (long c = (long)blockIdx.x * 256 + threadIdx.x; c < nc; c += (long)gridDim.x * 256) {
    const int i = int(c % G.n[0]), j = int((c / G.n[0]) % G.n[1]), k = int(c / ((long)G.n[0] * G.n[1]));
    const int f0 = fidx<0>(G, i, j, k), f1 = fidx<1>(G, i, j, k);
    float* a = in + c * (DIM + 1);
    float* t = tg + c * DIM;
    a[0] = float(double(r[f0]) * inv_s);
    a[1] = float(double(r[f1]) * inv_s);
    t[0] = float(double(et[f0]) * lam_over_s);
    t[1] = float(double(et[f1]) * lam_over_s);
    if (DIM == 3) {
      const int f2 = fidx<2>(G, i, j, k);
      a[2] = float(double(r[f2]) * inv_s);
      t[2] = float(double(et[f2]) * lam_over_s);
    }
    a[DIM] = logmu[c];
  }
}

// et = xs - xi - vr  (error of snapshot i after one V-cycle)
template <typename T>
__global__ __launch_bounds__(256) void k_err_after_v(int n, const T* __restrict__ xs,
                                                     const T* __restrict__ xi,
                                                     const T* __restrict__ vr, T* __restrict__ et) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) et[i] = xs[i] - xi[i] - vr[i];
}

}  // namespace gkb

namespace {

bool learned_enabled(Learned* L) { return L && L->net && !L->off; }
bool learned_has_net(Learned* L) { return L && L->net; }
void learned_reset(Learned* L) {
  if (L) {
    L->off = false;
    L->gain_sum = 0.0;
    L->gain_n = 0;
  }
}
bool learned_capturing(Learned* L) { return L && L->cap_in && L->cap_n < L->cap_max; }

int learned_create(gkb_ctx* c) {
  c->learned = new (std::nothrow) Learned();
  if (!c->learned) return GKB_ENOMEM;
  Learned* L = c->learned;
  long mf, nc, mu, nu;
  gkb_sizes(c, &mf, &nc, &mu, &nu);
  L->m_unknown = std::max<long>(mu, 1);
  CK(c->mem.arr(&L->logmu, c->g.n_cells));
  if (c->varmu) {
    std::vector<double> mh(c->g.n_cells);
    CK(copy_sync(c, mh.data(), c->coef64[0].mu, mh.size() * 8, hipMemcpyDeviceToHost));
    std::vector<float> lm(mh.size());
    for (size_t i = 0; i < mh.size(); ++i) lm[i] = float(std::log(mh[i]));
    CK(copy_sync(c, L->logmu, lm.data(), lm.size() * 4, hipMemcpyHostToDevice));
  }
  // lambda = mean of diag(W) over the unknown faces: the error a V-cycle
  // leaves behind is mostly divergence free, where M acts as W
  const size_t es = c->opt.precision == GKB_MIXED ? 4 : 8;
  {
    Op<double> opW = c->op64;
    opW.eta = 0.0;
    double* dw = nullptr;
    CK(c->mem.arr(&dw, c->g.m_full));
    face_op<double, kDiag>(c, opW, c->fl0, nullptr, nullptr, dw, 0.0, nullptr, nullptr);
    std::vector<double> dh(c->g.m_full);
    HIPCK(hipMemcpyAsync(dh.data(), dw, dh.size() * 8, hipMemcpyDeviceToHost, c->cs));
    HIPCK(hipStreamSynchronize(c->cs));
    double sum = 0.0;
    long cnt = 0;
    for (double v : dh)
      if (v != 0.0) {
        sum += v;
        ++cnt;
      }
    L->lam = cnt ? sum / cnt : 1.0;
  }
  CK(c->mem.get(&L->zv, c->g.m_full * es));
  CK(c->mem.get(&L->tmp, c->g.m_full * es));
  return GKB_OK;
}

void learned_destroy(gkb_ctx* c) {
  delete c->learned;
  c->learned = nullptr;
}

// z = V(r) + theta c for the residual r_in into z_out (c, M c and the
// post-V-cycle residual in scratch buffers).  st_dot: the flag that skips the
// launches (null: always run); st: the state that receives rt.rt, theta and
// the gain and whose done / fallback flags skip the network kernels.  In
// flexible CG r_in = in.r, z_out = in.z and k_combine also forms the dot
// partials of the direction choice; FGMRES passes its basis vector and
// preconditioned vector.
template <typename T>
void learned_apply(gkb_ctx* c, Inner<T>& in, const T* r_in, T* z_out, const PcgState* st_dot,
                   PcgState* st) {
  Learned* L = c->learned;
  const Level<T>& L0 = in.lv[0];
  const Grid& G = L0.g;
  gkb_cnn* net = L->net;
  T* zv = static_cast<T*>(L->zv);
  hipStream_t s = c->cs;
  // zv = V(r) with the partial r.zv; rt = r - M zv, the residual the V-cycle
  // leaves, is the network input (its scale from rt.rt)
  vcycle<T>(c, in, 0, r_in, zv, c->part[2], st_dot);
  T* rt = static_cast<T*>(L->tmp);
  face_op<T, kResidDot>(c, L0.op, L0.fl, zv, r_in, rt, T(0), c->part[1], st_dot);
  k_set_rt2<<<1, kFinal, 0, s>>>(st, c->part[1], L0.fl.nparts);
  const int nb = cnn_grid(G.n_cells);
  if (G.dim == 2)
    k_pack_faces<T, 2><<<nb, 256, 0, s>>>(G, rt, st, double(L->m_unknown), L->logmu, net->act[0]);
  else
    k_pack_faces<T, 3><<<nb, 256, 0, s>>>(G, rt, st, double(L->m_unknown), L->logmu, net->act[0]);
  CnnGeom g{G.n[0], G.n[1], G.n[2], 1, (long)G.n_cells};
  const int blocks = conv_blocks(g.P);
  const int* f1 = &st->done;
  const int* f2 = &st->fallback;
  for (int l = 0; l < net->L; ++l) {
    const uint16_t* w = net->wf + (size_t)l * net->taps * 256;
    const float* b = net->bias + 16 * l;
    const int cin = net->ch[l];
    if (G.dim == 2) {
      if (l < net->L - 1)
        launch_conv<2, kOutReluBf16>(cin, blocks, s, g, net->act[l], w, b, net->act[l + 1], nullptr, f1, f2);
      else
        launch_conv<2, kOutF32>(cin, blocks, s, g, net->act[l], w, b, net->y16, nullptr, f1, f2);
    } else {
      if (l < net->L - 1)
        launch_conv<3, kOutReluBf16>(cin, blocks, s, g, net->act[l], w, b, net->act[l + 1], nullptr, f1, f2);
      else
        launch_conv<3, kOutF32>(cin, blocks, s, g, net->act[l], w, b, net->y16, nullptr, f1, f2);
    }
  }
  // c (stored in z_out) with c.rt, then M c (into the rt buffer) with c.Mc,
  // the energy-optimal weight theta, and z = zv + theta c
  const dim3 tg = transfer_grid(G);
  if (G.dim == 2)
    k_unpack_c<T, 2><<<tg, 256, 0, s>>>(G, net->y16, st, double(L->m_unknown), L->lam, rt,
                                        z_out, c->part[3]);
  else
    k_unpack_c<T, 3><<<tg, 256, 0, s>>>(G, net->y16, st, double(L->m_unknown), L->lam, rt,
                                        z_out, c->part[3]);
  face_op<T, kApplyDot>(c, L0.op, L0.fl, z_out, nullptr, rt, T(0), c->part[4], st_dot);
  k_set_theta<<<1, kFinal, 0, s>>>(st, c->part[3], (int)(tg.x * tg.z), c->part[4],
                                   L0.fl.nparts);
  const int n = G.m_full;
  k_combine<T><<<vec_blocks(n), 256, 0, s>>>(n, st, zv, z_out, r_in, in.rprev, z_out, c->part[3],
                                             c->part[4], c->part[5]);
}

template <typename T>
void learned_precondition(gkb_ctx* c, Inner<T>& in, const PcgState* st_dot) {
  learned_apply<T>(c, in, in.r, in.z, st_dot, in.st);
}

template <typename T>
void fcg_iterations(gkb_ctx* c, Inner<T>& in, int count) {
  const Level<T>& L0 = in.lv[0];
  const int n = L0.g.m_full, vb = vec_blocks(n);
  const int nu = vb;  // partials of k_combine
  hipStream_t s = c->cs;
  T* zv = static_cast<T*>(c->learned->zv);
  for (int it = 0; it < count; ++it) {
    face_op<T, kApplyDot>(c, L0.op, L0.fl, in.p, nullptr, in.q, T(0), c->part[0], in.st);
    k_pcg_alpha<<<1, kFinal, 0, s>>>(in.st, c->part[0], L0.fl.nparts);
    k_fcg_xr<T><<<vb, 256, 0, s>>>(n, in.st, in.p, in.q, in.x, in.r, in.rprev, c->part[1]);
    k_pcg_check<<<1, kFinal, 0, s>>>(in.st, c->part[1], vb, nullptr, 0);
    learned_precondition<T>(c, in, in.st);
    k_fcg_beta<<<1, kFinal, 0, s>>>(in.st, c->part[2], vcycle_parts<T>(c, in), c->part[3],
                                    c->part[4], c->part[5], nu, 0, c->opt.learned_min_gain);
    k_fcg_p<T><<<vb, 256, 0, s>>>(n, in.st, in.z, zv, in.p);
  }
}

// network buffers for the grid and BF16 weights from the current FP32 ones
int learned_prepare(gkb_ctx* c) {
  gkb_cnn* net = c->learned->net;
  CK(cnn_reserve(net, c->g.n_cells));
  CK(cnn_prepare_weights(net));
  HIPCK(hipStreamSynchronize(net->s));
  return GKB_OK;
}

template <typename T>
int learned_solve(gkb_ctx* c, const double* f, double* x_out, double tol, int* iters) {
  Inner<T>& in = inner_of<T>(c);
  Learned* L = c->learned;
  gkb_cnn* net = L->net;
  const Level<T>& L0 = in.lv[0];
  const Grid& G = L0.g;
  const int n = G.m_full, vb = vec_blocks(n);
  const int nu = vb;  // partials of k_combine
  hipStream_t s = c->cs;
  CK(cnn_reserve(net, G.n_cells));
  CK(cnn_prepare_weights(net));
  HIPCK(hipStreamSynchronize(net->s));
  T* zv = static_cast<T*>(L->zv);
  k_pcg_init<double, T><<<vb, kBlock, 0, s>>>(n, f, in.x, in.r, c->part[3]);
  k_fill<T><<<vb, kBlock, 0, s>>>(n, T(0), in.rprev);
  k_pcg_start<<<1, kFinal, 0, s>>>(in.st, c->part[3], vb, c->part[3], vb, tol, c->opt.inner_maxit);
  learned_precondition<T>(c, in, nullptr);
  k_fcg_beta<<<1, kFinal, 0, s>>>(in.st, c->part[2], vcycle_parts<T>(c, in), c->part[3], c->part[4],
                                  c->part[5], nu, 1, c->opt.learned_min_gain);
  k_fill<T><<<vb, kBlock, 0, s>>>(n, T(0), in.p);
  k_fcg_p<T><<<vb, 256, 0, s>>>(n, in.st, in.z, zv, in.p);
  PcgState hs;
  // a network that fails the guards at its first application is not used for
  // this solve (plain MG-PCG has no flexible-CG overhead), nor for the rest
  // of the gkb_solve
  HIPCK(hipMemcpyAsync(c->hbuf, in.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  std::memcpy(&hs, c->hbuf, sizeof(PcgState));
  if (hs.fallback) {
    c->stats.learned_solves += 1;
    c->stats.fallbacks += 1;
    L->gain_sum += hs.gain_sum;
    L->gain_n += hs.gain_n;
    c->stats.learned_gain = L->gain_n ? L->gain_sum / L->gain_n : -1.0;
    L->off = true;
    c->stats.learned_fallback_reason = hs.fb_reason;
    c->stats.learned_fallback_iteration = hs.fb_it;
    return kLearnedDeclined;
  }
  const int chunk = std::max(1, c->opt.check_every);
  if (c->opt.use_graphs) {
    if (!(in.graph_fcg && in.graph_fcg_len == chunk)) {
      if (in.graph_fcg) (void)hipGraphExecDestroy(in.graph_fcg);
      in.graph_fcg = nullptr;
      hipGraph_t gr;
      HIPCK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      fcg_iterations<T>(c, in, chunk);
      HIPCK(hipStreamEndCapture(s, &gr));
      HIPCK(hipGraphInstantiate(&in.graph_fcg, gr, nullptr, nullptr, 0));
      (void)hipGraphDestroy(gr);
      in.graph_fcg_len = chunk;
    }
  }
  for (;;) {
    if (c->opt.use_graphs) HIPCK(hipGraphLaunch(in.graph_fcg, s));
    else fcg_iterations<T>(c, in, chunk);
    HIPCK(hipMemcpyAsync(c->hbuf, in.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    std::memcpy(&hs, c->hbuf, sizeof(PcgState));
    if (hs.done) break;
    if (hs.fallback && !hs.nonfinite) {
      // the network failed a guard during the solve: its flexible-CG iterates
      // are dropped and plain MG-PCG solves from scratch (a direction the
      // network spoiled can slow the rest of a flexible-CG solve a lot)
      c->stats.inner_iterations += hs.it;
      c->stats.learned_solves += 1;
      c->stats.fallbacks += hs.fallbacks;
      L->gain_sum += hs.gain_sum;
      L->gain_n += hs.gain_n;
      c->stats.learned_gain = L->gain_n ? L->gain_sum / L->gain_n : -1.0;
      L->off = true;
      c->stats.learned_fallback_reason = hs.fb_reason;
      c->stats.learned_fallback_iteration = hs.fb_it;
      return kLearnedDeclined;
    }
  }
  k_cast<T, double><<<vb, kBlock, 0, s>>>(n, in.x, x_out);
  if (hs.fallbacks > 0) {
    c->stats.learned_fallback_reason = hs.fb_reason;
    c->stats.learned_fallback_iteration = hs.fb_it;
  }
  if (iters) *iters = hs.it;
  c->stats.inner_iterations += hs.it;
  c->stats.inner_solves += 1;
  c->stats.learned_solves += 1;
  c->stats.fallbacks += hs.fallbacks;
  L->gain_sum += hs.gain_sum;
  L->gain_n += hs.gain_n;
  c->stats.learned_gain = L->gain_n ? L->gain_sum / L->gain_n : -1.0;
  if (hs.fallbacks > 0) L->off = true;
  if (hs.nonfinite) return GKB_ENAN;
  if (hs.status == -5) return GKB_EINNER;
  return GKB_OK;
}

// MG-PCG inner solve that records training pairs (no graph: snapshots are
// taken between iterations)
template <typename T>
int capture_solve(gkb_ctx* c, const double* f, double* x_out, double tol, int* iters) {
  Inner<T>& in = inner_of<T>(c);
  Learned* L = c->learned;
  const Level<T>& L0 = in.lv[0];
  const Grid& G = L0.g;
  const int n = G.m_full, vb = vec_blocks(n);
  hipStream_t s = c->cs;
  const int ns = (int)L->cap_iters.size();
  if ((int)L->snaps.size() < 2 * ns) {
    for (int k = (int)L->snaps.size(); k < 2 * ns; ++k) {
      void* p = nullptr;
      CK(c->mem.get(&p, (size_t)n * sizeof(T)));
      L->snaps.push_back(p);
    }
  }
  k_pcg_init<double, T><<<vb, kBlock, 0, s>>>(n, f, in.x, in.r, c->part[3]);
  vcycle<T>(c, in, 0, in.r, in.z, nullptr, nullptr);
  k_pcg_p0<T><<<vb, kBlock, 0, s>>>(n, nullptr, in.r, in.z, in.p, c->part[2]);
  k_pcg_start<<<1, kFinal, 0, s>>>(in.st, c->part[3], vb, c->part[2], vb, tol, c->opt.inner_maxit);
  std::vector<char> taken(ns, 0);
  PcgState hs;
  int it = 0;
  for (;;) {
    for (int k = 0; k < ns; ++k)
      if (!taken[k] && L->cap_iters[k] == it) {
        k_cast<T, T><<<vb, kBlock, 0, s>>>(n, in.r, static_cast<T*>(L->snaps[2 * k]));
        k_cast<T, T><<<vb, kBlock, 0, s>>>(n, in.x, static_cast<T*>(L->snaps[2 * k + 1]));
        taken[k] = 1;
      }
    CK(pcg_iterations<T>(c, in, 1));
    HIPCK(hipMemcpyAsync(c->hbuf, in.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    std::memcpy(&hs, c->hbuf, sizeof(PcgState));
    ++it;
    if (hs.done) break;
  }
  T* tmp = static_cast<T*>(L->tmp);
  for (int k = 0; k < ns && L->cap_n < L->cap_max; ++k) {
    if (!taken[k]) continue;
    T* rk = static_cast<T*>(L->snaps[2 * k]);
    T* xk = static_cast<T*>(L->snaps[2 * k + 1]);
    // input: rt = r_k - M V(r_k); target: x* - x_k - V(r_k)
    vcycle<T>(c, in, 0, rk, in.z, nullptr, nullptr);
    T* rt = in.q;
    face_op<T, kResid>(c, L0.op, L0.fl, in.z, rk, rt, T(0), nullptr, nullptr);
    k_dot<T><<<vb, kBlock, 0, s>>>(n, rt, rt, c->part[0]);
    double rr = 0.0;
    CK(host_sum(c, c->part[0], vb, &rr));
    if (!(rr > 0.0)) continue;
    const double sr = std::sqrt(rr / double(L->m_unknown));
    k_err_after_v<T><<<vb, kBlock, 0, s>>>(n, in.x, xk, in.z, tmp);
    const long nc = G.n_cells;
    float* pin = L->cap_in + (size_t)L->cap_n * nc * (G.dim + 1);
    float* ptg = L->cap_tg + (size_t)L->cap_n * nc * G.dim;
    if (G.dim == 2)
      k_pack_pair<T, 2><<<cnn_grid(nc), 256, 0, s>>>(G, rt, tmp, 1.0 / sr, L->lam / sr, L->logmu, pin, ptg);
    else
      k_pack_pair<T, 3><<<cnn_grid(nc), 256, 0, s>>>(G, rt, tmp, 1.0 / sr, L->lam / sr, L->logmu, pin, ptg);
    L->cap_n += 1;
  }
  k_cast<T, double><<<vb, kBlock, 0, s>>>(n, in.x, x_out);
  HIPCK(hipStreamSynchronize(s));
  if (iters) *iters = hs.it;
  c->stats.inner_iterations += hs.it;
  c->stats.inner_solves += 1;
  if (hs.nonfinite) return GKB_ENAN;
  if (hs.status == -5) return GKB_EINNER;
  return GKB_OK;
}

}  // namespace

extern "C" {

int gkb_attach_cnn(gkb_ctx* c, gkb_cnn* net) {
  if (!c || !c->learned) return GKB_EINVAL;
  if (net) {
    if (net->dim != c->g.dim || net->ch[0] != c->g.dim + 1 || net->ch[net->L] != c->g.dim)
      return GKB_EINVAL;
    CK(cnn_reserve(net, c->g.n_cells));
  }
  c->learned->net = net;
  // the flexible-CG and FGMRES graphs hold the network's buffers; the PCG
  // graphs do not
  if (c->in32.graph_fcg) (void)hipGraphExecDestroy(c->in32.graph_fcg);
  if (c->in64.graph_fcg) (void)hipGraphExecDestroy(c->in64.graph_fcg);
  if (c->in32.graph_gm) (void)hipGraphExecDestroy(c->in32.graph_gm);
  if (c->in64.graph_gm) (void)hipGraphExecDestroy(c->in64.graph_gm);
  c->in32.graph_fcg = nullptr;
  c->in64.graph_fcg = nullptr;
  c->in32.graph_gm = nullptr;
  c->in64.graph_gm = nullptr;
  return GKB_OK;
}

int gkb_set_capture(gkb_ctx* c, float* inputs, float* targets, int max_pairs, int n_iters,
                    const int* iters) {
  if (!c || !c->learned) return GKB_EINVAL;
  Learned* L = c->learned;
  if (!inputs) {
    L->cap_in = L->cap_tg = nullptr;
    L->cap_max = 0;
    return GKB_OK;
  }
  if (!targets || max_pairs < 1 || n_iters < 1 || n_iters > 16 || !iters) return GKB_EINVAL;
  L->cap_in = inputs;
  L->cap_tg = targets;
  L->cap_max = max_pairs;
  L->cap_n = 0;
  L->cap_iters.assign(iters, iters + n_iters);
  return GKB_OK;
}

int gkb_capture_count(const gkb_ctx* c, int* count) {
  if (!c || !c->learned || !count) return GKB_EINVAL;
  *count = c->learned->cap_n;
  return GKB_OK;
}

}  // extern "C"
