// Host side of the learned warm start (included at the end of pdlp.hip, after the solver and the
// problem / batch handles): parameter store, Adam state, per-graph workspace, the forward and
// backward launch sequences, and the pdlp_gnn_* entry points declared in include/pdlp_gnn.h.
#pragma once
#include <random>

#include "../../include/pdlp_gnn.h"
#include "gnn_kernels.h"

namespace pdlp {
namespace gnn {

// Flat parameter layout (FP32): Wv_in [8x64], bv_in, Wc_in [8x64], bc_in, then per layer
// W1, W2 [64x64], b1, W3, W4 [64x64], b3, then wx, bx, wy, by, wov, woc, bo. Matrices row-major
// [input channel][output channel].
constexpr int64_t kOffWvIn = 0, kOffBvIn = 512, kOffWcIn = 576, kOffBcIn = 1088, kOffLayer0 = 1152;
constexpr int64_t kLayerStride = 2 * 4096 + 64 + 2 * 4096 + 64;
constexpr int64_t off_W1(int l) { return kOffLayer0 + l * kLayerStride; }
constexpr int64_t off_W2(int l) { return off_W1(l) + 4096; }
constexpr int64_t off_b1(int l) { return off_W1(l) + 8192; }
constexpr int64_t off_W3(int l) { return off_W1(l) + 8256; }
constexpr int64_t off_W4(int l) { return off_W1(l) + 12352; }
constexpr int64_t off_b3(int l) { return off_W1(l) + 16448; }
constexpr int64_t kOffHeads = kOffLayer0 + kLayers * kLayerStride;
constexpr int64_t kOffWx = kOffHeads, kOffBx = kOffWx + 64, kOffWy = kOffBx + 1, kOffBy = kOffWy + 64;
constexpr int64_t kOffWov = kOffBy + 1, kOffWoc = kOffWov + 64, kOffBo = kOffWoc + 64;
constexpr int64_t kNumParams = kOffBo + 1;
static_assert(kNumParams == 50947, "parameter count");

constexpr int kMaxWavesBwd = 512;
constexpr int kMaxWavesFwd = 2048;

// The scaled, renumbered problem of a solver handle as the network reads it.
struct GraphView {
  int32_t K = 0, m = 0, n = 0, nnz = 0;
  std::vector<int32_t> h_row0, h_col0;
  const int32_t *row0 = nullptr, *col0 = nullptr;
  const int32_t *a_rp = nullptr, *a_ci = nullptr, *t_rp = nullptr, *t_ci = nullptr;
  const float *a_v = nullptr, *t_v = nullptr;        // FP32 values (null for an FP64 handle)
  const double *a_v64 = nullptr, *t_v64 = nullptr;
  const double *c = nullptr, *b = nullptr, *l = nullptr, *u = nullptr, *Dr = nullptr, *Dc = nullptr;
  const uint8_t *sense = nullptr;
  const int32_t *perm_r = nullptr, *perm_c = nullptr, *inv_r = nullptr, *inv_c = nullptr;
  hipStream_t stream = nullptr;
};

template <typename T>
GraphView view_of(Solver<T> &s) {
  GraphView g;
  g.K = s.K, g.m = s.m, g.n = s.n, g.nnz = s.nnz;
  g.h_row0 = s.h_row0, g.h_col0 = s.h_col0;
  g.row0 = s.d_row0, g.col0 = s.d_col0;
  g.a_rp = s.a_rp, g.a_ci = s.a_ci, g.t_rp = s.t_rp, g.t_ci = s.t_ci;
  if constexpr (sizeof(T) == sizeof(float)) g.a_v = s.a_v, g.t_v = s.t_v;
  g.a_v64 = s.a_v64, g.t_v64 = s.t_v64;
  g.c = s.c64, g.b = s.b64, g.l = s.l64, g.u = s.u64, g.Dr = s.Dr, g.Dc = s.Dc;
  g.sense = s.sense;
  g.perm_r = s.d_perm_r, g.perm_c = s.d_perm_c, g.inv_r = s.d_inv_r, g.inv_c = s.d_inv_c;
  g.stream = s.stream;
  return g;
}

inline int grid_cap(int64_t work, int per_block, int cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((work + per_block - 1) / per_block, cap));
}

struct Model {
  Arena mem;  // parameters and optimiser state
  float *P = nullptr, *G = nullptr, *M1 = nullptr, *M2 = nullptr;
  int64_t step = 0;
  float omega_weight = 1.f;  // weight of the log-omega term of the loss
  // per-graph workspace, regrown when a larger graph arrives
  Arena ws;
  int64_t cap_n = -1, cap_m = -1, cap_nnz = -1, cap_k = -1, cap_chv = -1, cap_chc = -1;
  float *fv, *fc, *hv[kLayers + 1], *hc[kLayers + 1], *mv[kLayers], *mc[kLayers];
  float *dhv[2], *dhc[2], *dmv, *dmc, *part, *gpart_v, *gpart_c;
  float *xhat, *yhat, *logw, *pv, *pc, *vpool, *cpool, *dlw, *tx, *ty, *tw, *a_v32, *t_v32;
  double *vsq, *csq, *lossq, *ext_n, *ext_m;
  int32_t *vcs, *vce, *vcq, *ccs, *cce, *ccq, *vch0, *cch0;
  // chunk tables of the current graph (host)
  std::vector<int32_t> h_vcs, h_vce, h_vcq, h_ccs, h_cce, h_ccq, h_vch0, h_cch0;

  void init(uint64_t seed) {
    P = mem.alloc<float>(kNumParams), G = mem.alloc<float>(kNumParams);
    M1 = mem.alloc<float>(kNumParams), M2 = mem.alloc<float>(kNumParams);
    std::vector<float> h((size_t)kNumParams, 0.f);
    std::mt19937_64 rng(seed);
    auto glorot = [&](int64_t off, int fan_in, int fan_out) {
      const double lim = std::sqrt(6.0 / (fan_in + fan_out));
      std::uniform_real_distribution<double> U(-lim, lim);
      for (int64_t e = 0; e < (int64_t)fan_in * fan_out; ++e) h[(size_t)(off + e)] = (float)U(rng);
    };
    glorot(kOffWvIn, kF, kH);
    glorot(kOffWcIn, kF, kH);
    for (int l = 0; l < kLayers; ++l) {
      glorot(off_W1(l), kH, kH), glorot(off_W2(l), kH, kH);
      glorot(off_W3(l), kH, kH), glorot(off_W4(l), kH, kH);
    }
    glorot(kOffWx, kH, 1), glorot(kOffWy, kH, 1), glorot(kOffWov, kH, 1), glorot(kOffWoc, kH, 1);
    set_params(h.data(), nullptr);
  }

  void set_params(const float *host, hipStream_t st) {
    HIPCHK(hipMemcpy(P, host, sizeof(float) * kNumParams, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(M1, 0, sizeof(float) * kNumParams));
    HIPCHK(hipMemset(M2, 0, sizeof(float) * kNumParams));
    HIPCHK(hipMemset(G, 0, sizeof(float) * kNumParams));
    step = 0;
    (void)st;
  }

  void build_chunks(const GraphView &g) {
    auto side = [&](const std::vector<int32_t> &off, std::vector<int32_t> &cs, std::vector<int32_t> &ce,
                    std::vector<int32_t> &cq, std::vector<int32_t> &ch0) {
      cs.clear(), ce.clear(), cq.clear(), ch0.assign(1, 0);
      for (int32_t q = 0; q < g.K; ++q) {
        for (int32_t s = off[q]; s < off[q + 1]; s += kChunk)
          cs.push_back(s), ce.push_back(std::min(s + kChunk, off[q + 1])), cq.push_back(q);
        ch0.push_back((int32_t)cs.size());
      }
    };
    side(g.h_col0, h_vcs, h_vce, h_vcq, h_vch0);
    side(g.h_row0, h_ccs, h_cce, h_ccq, h_cch0);
  }

  // Workspace for the graph. Prediction keeps two activation buffers and one message buffer per
  // side (the layers alternate between them); training keeps every layer for the backward pass and
  // the gradient buffers (about 14 x 64 floats per node against 3 x 64).
  bool cap_train = false;
  void ensure(const GraphView &g, bool training) {
    const int64_t nchv = (int64_t)h_vcs.size(), nchc = (int64_t)h_ccs.size();
    const bool need_vals = g.a_v == nullptr;
    if (g.n <= cap_n && g.m <= cap_m && g.K <= cap_k && nchv <= cap_chv && nchc <= cap_chc &&
        (!need_vals || g.nnz <= cap_nnz) && (!training || cap_train))
      return;
    ws.reset();
    cap_train = cap_train || training;
    cap_n = std::max<int64_t>(g.n, cap_n), cap_m = std::max<int64_t>(g.m, cap_m);
    cap_k = std::max<int64_t>(g.K, cap_k), cap_chv = std::max(nchv, cap_chv), cap_chc = std::max(nchc, cap_chc);
    cap_nnz = std::max<int64_t>(need_vals ? g.nnz : 0, cap_nnz);
    const int64_t N = cap_n, M = cap_m;
    fv = ws.alloc<float>(N * kF), fc = ws.alloc<float>(M * kF);
    if (cap_train) {
      for (int l = 0; l <= kLayers; ++l) hv[l] = ws.alloc<float>(N * kH), hc[l] = ws.alloc<float>(M * kH);
      for (int l = 0; l < kLayers; ++l) mv[l] = ws.alloc<float>(N * kH), mc[l] = ws.alloc<float>(M * kH);
      for (int t = 0; t < 2; ++t) dhv[t] = ws.alloc<float>(N * kH), dhc[t] = ws.alloc<float>(M * kH);
      dmv = ws.alloc<float>(N * kH), dmc = ws.alloc<float>(M * kH);
      part = ws.alloc<float>((int64_t)kMaxWavesBwd * (kH * kH * 2 + kH));
    } else {
      float *v2[2] = {ws.alloc<float>(N * kH), ws.alloc<float>(N * kH)};
      float *c2[2] = {ws.alloc<float>(M * kH), ws.alloc<float>(M * kH)};
      float *mv1 = ws.alloc<float>(N * kH), *mc1 = ws.alloc<float>(M * kH);
      for (int l = 0; l <= kLayers; ++l) hv[l] = v2[l & 1], hc[l] = c2[l & 1];
      for (int l = 0; l < kLayers; ++l) mv[l] = mv1, mc[l] = mc1;
      dhv[0] = dhv[1] = dhc[0] = dhc[1] = dmv = dmc = part = nullptr;
    }
    gpart_v = ws.alloc<float>(cap_chv * (kH + 1)), gpart_c = ws.alloc<float>(cap_chc * (kH + 1));
    xhat = ws.alloc<float>(N), yhat = ws.alloc<float>(M), tx = ws.alloc<float>(N), ty = ws.alloc<float>(M);
    logw = ws.alloc<float>(cap_k), tw = ws.alloc<float>(cap_k), dlw = ws.alloc<float>(cap_k);
    pv = ws.alloc<float>(cap_k * kH), pc = ws.alloc<float>(cap_k * kH);
    vpool = ws.alloc<float>(cap_chv * kH), cpool = ws.alloc<float>(cap_chc * kH);
    vsq = ws.alloc<double>(cap_chv), csq = ws.alloc<double>(cap_chc), lossq = ws.alloc<double>(cap_k);
    ext_n = ws.alloc<double>(N), ext_m = ws.alloc<double>(M);
    vcs = ws.alloc<int32_t>(cap_chv), vce = ws.alloc<int32_t>(cap_chv), vcq = ws.alloc<int32_t>(cap_chv);
    ccs = ws.alloc<int32_t>(cap_chc), cce = ws.alloc<int32_t>(cap_chc), ccq = ws.alloc<int32_t>(cap_chc);
    vch0 = ws.alloc<int32_t>(cap_k + 1), cch0 = ws.alloc<int32_t>(cap_k + 1);
    a_v32 = t_v32 = nullptr;
    if (cap_nnz > 0) a_v32 = ws.alloc<float>(cap_nnz), t_v32 = ws.alloc<float>(cap_nnz);
  }

  // Upload chunk tables, FP32 values when the handle iterates in FP64. Returns the value arrays.
  void prepare(const GraphView &g, const float *&av, const float *&tv, bool training) {
    build_chunks(g);
    ensure(g, training);
    hipStream_t st = g.stream;
    auto up = [&](int32_t *d, const std::vector<int32_t> &h) {
      if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, st));
    };
    up(vcs, h_vcs), up(vce, h_vce), up(vcq, h_vcq), up(ccs, h_ccs), up(cce, h_cce), up(ccq, h_ccq);
    up(vch0, h_vch0), up(cch0, h_cch0);
    if (g.a_v) {
      av = g.a_v, tv = g.t_v;
    } else {
      if (g.nnz > 0) {
        hipLaunchKernelGGL(g_to_float, dim3(grid_cap(g.nnz, kGB, 4096)), dim3(kGB), 0, st, (int64_t)g.nnz,
                           g.a_v64, a_v32);
        hipLaunchKernelGGL(g_to_float, dim3(grid_cap(g.nnz, kGB, 4096)), dim3(kGB), 0, st, (int64_t)g.nnz,
                           g.t_v64, t_v32);
      }
      av = a_v32, tv = t_v32;
    }
  }

  template <int K1, bool TWO>
  void dense_fwd(hipStream_t st, int32_t R, const float *X1, int64_t w1, const float *X2, int64_t w2, int64_t bias,
                 float *out) {
    if (R <= 0) return;
    const int waves = grid_cap((R + 15) / 16, 1, kMaxWavesFwd);
    hipLaunchKernelGGL((g_dense_fwd<K1, TWO>), dim3((waves + 3) / 4), dim3(kGB), 0, st, R, X1, P + w1, X2,
                       TWO ? P + w2 : nullptr, P + bias, out);
  }

  // backward of one dense layer; the parameter gradient block starting at w1 gets K1*64 (+4096) + 64
  template <int K1, bool TWO, bool DX1>
  void dense_bwd(hipStream_t st, int32_t R, const float *out, const float *dout, const float *X1, int64_t w1,
                 const float *X2, int64_t w2, float *dX1, float *dX2) {
    constexpr int LEN = K1 * kH + (TWO ? kH * kH : 0) + kH;
    if (R <= 0) {
      HIPCHK(hipMemsetAsync(G + w1, 0, sizeof(float) * LEN, st));
      return;
    }
    const int blocks = (grid_cap((R + 15) / 16, 1, kMaxWavesBwd) + 3) / 4;
    hipLaunchKernelGGL((g_dense_bwd<K1, TWO, DX1>), dim3(blocks), dim3(kGB), 0, st, R, out, dout, X1, P + w1, X2,
                       TWO ? P + w2 : nullptr, dX1, dX2, part);
    hipLaunchKernelGGL(g_reduce_waves, dim3((LEN + kGB - 1) / kGB), dim3(kGB), 0, st, blocks * 4, LEN,
                       (const float *)part, G + w1);
  }

  template <bool ACC>
  void spmm(hipStream_t st, int32_t R, const int32_t *rp, const int32_t *ci, const float *v, const float *in,
            float *out) {
    if (R <= 0) return;
    hipLaunchKernelGGL(g_spmm<ACC>, dim3(grid_cap(R, kGB / 16, 65536)), dim3(kGB), 0, st, R, rp, ci, v, in, out);
  }

  // Forward pass over the whole graph; with targets also the loss terms (tx, ty, tw loaded).
  void forward(const GraphView &g, const float *av, const float *tv, bool with_targets) {
    hipStream_t st = g.stream;
    const int32_t n = g.n, m = g.m;
    if (n + m > 0)
      hipLaunchKernelGGL(g_features, dim3(grid_cap(n + m, kGB, 8192)), dim3(kGB), 0, st, m, n, g.c, g.l, g.u,
                         g.t_rp, g.b, g.sense, g.a_rp, fv, fc);
    dense_fwd<kF, false>(st, n, fv, kOffWvIn, nullptr, 0, kOffBvIn, hv[0]);
    dense_fwd<kF, false>(st, m, fc, kOffWcIn, nullptr, 0, kOffBcIn, hc[0]);
    for (int l = 0; l < kLayers; ++l) {
      spmm<false>(st, m, g.a_rp, g.a_ci, av, hv[l], mc[l]);
      dense_fwd<kH, true>(st, m, hc[l], off_W1(l), mc[l], off_W2(l), off_b1(l), hc[l + 1]);
      spmm<false>(st, n, g.t_rp, g.t_ci, tv, hc[l + 1], mv[l]);
      dense_fwd<kH, true>(st, n, hv[l], off_W3(l), mv[l], off_W4(l), off_b3(l), hv[l + 1]);
    }
    const int nchv = (int)h_vcs.size(), nchc = (int)h_ccs.size();
    if (nchv)
      hipLaunchKernelGGL(g_head_fwd, dim3(nchv), dim3(kGB), 0, st, (const int32_t *)vcs, (const int32_t *)vce,
                         (const float *)hv[kLayers], (const float *)(P + kOffWx), (const float *)(P + kOffBx),
                         with_targets ? (const float *)tx : nullptr, xhat, vpool, vsq);
    if (nchc)
      hipLaunchKernelGGL(g_head_fwd, dim3(nchc), dim3(kGB), 0, st, (const int32_t *)ccs, (const int32_t *)cce,
                         (const float *)hc[kLayers], (const float *)(P + kOffWy), (const float *)(P + kOffBy),
                         with_targets ? (const float *)ty : nullptr, yhat, cpool, csq);
    hipLaunchKernelGGL(g_head_inst, dim3(g.K), dim3(64), 0, st, g.K, g.col0, g.row0, (const int32_t *)vch0,
                       (const int32_t *)cch0, (const float *)vpool, (const float *)cpool, (const double *)vsq,
                       (const double *)csq, (const float *)(P + kOffWov), (const float *)(P + kOffWoc),
                       (const float *)(P + kOffBo), with_targets ? (const float *)tw : nullptr, omega_weight, pv, pc,
                       logw, lossq, dlw);
    HIPCHK(hipGetLastError());
  }

  // Backward pass after forward(with_targets = true): fills G.
  void backward(const GraphView &g, const float *av, const float *tv) {
    hipStream_t st = g.stream;
    const int32_t n = g.n, m = g.m;
    const int nchv = (int)h_vcs.size(), nchc = (int)h_ccs.size();
    if (nchv)
      hipLaunchKernelGGL(g_head_bwd, dim3(nchv), dim3(kGB), 0, st, g.K, (const int32_t *)vcs, (const int32_t *)vce,
                         (const int32_t *)vcq, g.col0, (const float *)hv[kLayers], (const float *)xhat,
                         (const float *)tx, (const float *)(P + kOffWx), (const float *)(P + kOffWov),
                         (const float *)dlw, dhv[0], gpart_v);
    if (nchc)
      hipLaunchKernelGGL(g_head_bwd, dim3(nchc), dim3(kGB), 0, st, g.K, (const int32_t *)ccs, (const int32_t *)cce,
                         (const int32_t *)ccq, g.row0, (const float *)hc[kLayers], (const float *)yhat,
                         (const float *)ty, (const float *)(P + kOffWy), (const float *)(P + kOffWoc),
                         (const float *)dlw, dhc[0], gpart_c);
    hipLaunchKernelGGL(g_head_fin, dim3(1), dim3(64), 0, st, nchv, (const float *)gpart_v, g.K, (const float *)pv,
                       (const float *)dlw, G + kOffWx, G + kOffBx, G + kOffWov, G + kOffBo);
    hipLaunchKernelGGL(g_head_fin, dim3(1), dim3(64), 0, st, nchc, (const float *)gpart_c, g.K, (const float *)pc,
                       (const float *)dlw, G + kOffWy, G + kOffBy, G + kOffWoc, (float *)nullptr);
    int cur = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
      // variable side: hv[l+1] = relu(hv[l] W3 + mv W4 + b3)
      dense_bwd<kH, true, true>(st, n, hv[l + 1], dhv[cur], hv[l], off_W3(l), mv[l], off_W4(l), dhv[1 - cur], dmv);
      // mv = A' hc[l+1]  =>  dhc[l+1] += A dmv
      spmm<true>(st, m, g.a_rp, g.a_ci, av, dmv, dhc[cur]);
      // constraint side: hc[l+1] = relu(hc[l] W1 + mc W2 + b1)
      dense_bwd<kH, true, true>(st, m, hc[l + 1], dhc[cur], hc[l], off_W1(l), mc[l], off_W2(l), dhc[1 - cur], dmc);
      // mc = A hv[l]  =>  dhv[l] += A' dmc
      spmm<true>(st, n, g.t_rp, g.t_ci, tv, dmc, dhv[1 - cur]);
      cur = 1 - cur;
    }
    dense_bwd<kF, false, false>(st, n, hv[0], dhv[cur], fv, kOffWvIn, nullptr, 0, nullptr, nullptr);
    dense_bwd<kF, false, false>(st, m, hc[0], dhc[cur], fc, kOffWcIn, nullptr, 0, nullptr, nullptr);
    HIPCHK(hipGetLastError());
  }

  void load_targets(const GraphView &g, const double *x_star, const double *y_star, const double *omega_star) {
    hipStream_t st = g.stream;
    for (int32_t q = 0; q < g.K; ++q)
      if (!(omega_star[q] > 0.0) || !std::isfinite(omega_star[q])) raise(PDLP_ERR_ARG, "omega_star must be positive");
    if (g.n) {
      HIPCHK(hipMemcpyAsync(ext_n, x_star, sizeof(double) * (size_t)g.n, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(g_target, dim3(grid_cap(g.n, kGB, 4096)), dim3(kGB), 0, st, g.n, (const double *)ext_n,
                         g.perm_c, g.Dc, tx);
    }
    if (g.m) {
      HIPCHK(hipMemcpyAsync(ext_m, y_star, sizeof(double) * (size_t)g.m, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(g_target, dim3(grid_cap(g.m, kGB, 4096)), dim3(kGB), 0, st, g.m, (const double *)ext_m,
                         g.perm_r, g.Dr, ty);
    }
    std::vector<float> h((size_t)g.K);
    for (int32_t q = 0; q < g.K; ++q) h[q] = (float)std::log(omega_star[q]);
    HIPCHK(hipMemcpyAsync(tw, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // h goes out of scope
  }

  double loss(const GraphView &g) {
    std::vector<double> lq((size_t)g.K);
    HIPCHK(hipMemcpyAsync(lq.data(), lossq, sizeof(double) * lq.size(), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    double s = 0.0;
    for (double v : lq) s += v;
    return s / g.K;
  }
};

}  // namespace gnn
}  // namespace pdlp

struct pdlp_gnn {
  pdlp::gnn::Model model;
};

using pdlp::raise;  // for HIPCHK at file scope (overloads the C library's one-argument raise)

namespace {
template <typename F>
int with_graph(pdlp_gnn *g, pdlp::AnySolver &s, F &&fn) {
  return guarded([&] {
    s.visit([&](auto &solver) {
      pdlp::gnn::GraphView v = pdlp::gnn::view_of(solver);
      fn(v);
    });
  });
}

void gnn_predict(pdlp::gnn::Model &M, const pdlp::gnn::GraphView &v, double *x0, double *y0, double *omega0,
                 float *raw_x, float *raw_y, float *raw_logw) {
  using namespace pdlp::gnn;
  const float *av = nullptr, *tv = nullptr;
  M.prepare(v, av, tv, false);
  M.forward(v, av, tv, false);
  hipStream_t st = v.stream;
  if (x0 && v.n) {
    hipLaunchKernelGGL(g_unscale_pred, dim3(grid_cap(v.n, kGB, 4096)), dim3(kGB), 0, st, v.n, (const float *)M.xhat,
                       v.inv_c, v.Dc, M.ext_n);
    HIPCHK(hipMemcpyAsync(x0, M.ext_n, sizeof(double) * (size_t)v.n, hipMemcpyDeviceToHost, st));
  }
  if (y0 && v.m) {
    hipLaunchKernelGGL(g_unscale_pred, dim3(grid_cap(v.m, kGB, 4096)), dim3(kGB), 0, st, v.m, (const float *)M.yhat,
                       v.inv_r, v.Dr, M.ext_m);
    HIPCHK(hipMemcpyAsync(y0, M.ext_m, sizeof(double) * (size_t)v.m, hipMemcpyDeviceToHost, st));
  }
  if (raw_x && v.n) HIPCHK(hipMemcpyAsync(raw_x, M.xhat, sizeof(float) * (size_t)v.n, hipMemcpyDeviceToHost, st));
  if (raw_y && v.m) HIPCHK(hipMemcpyAsync(raw_y, M.yhat, sizeof(float) * (size_t)v.m, hipMemcpyDeviceToHost, st));
  std::vector<float> lw((size_t)v.K);
  HIPCHK(hipMemcpyAsync(lw.data(), M.logw, sizeof(float) * lw.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int32_t q = 0; q < v.K; ++q) {
    if (raw_logw) raw_logw[q] = lw[q];
    if (omega0) omega0[q] = std::exp(std::min(20.0, std::max(-20.0, (double)lw[q])));
  }
}
}  // namespace

extern "C" {

int64_t pdlp_gnn_num_params(void) { return pdlp::gnn::kNumParams; }

int pdlp_gnn_create(pdlp_gnn **out, uint64_t seed) {
  if (!out) {
    pdlp::g_last_error = "out is NULL";
    return PDLP_ERR_ARG;
  }
  *out = nullptr;
  return guarded([&] {
    auto g = std::make_unique<pdlp_gnn>();
    g->model.init(seed);
    *out = g.release();
  });
}

int pdlp_gnn_get_params(pdlp_gnn *g, float *params) {
  if (!g || !params) {
    pdlp::g_last_error = "bad argument to pdlp_gnn_get_params";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(params, g->model.P, sizeof(float) * pdlp::gnn::kNumParams, hipMemcpyDeviceToHost));
  });
}

int pdlp_gnn_set_params(pdlp_gnn *g, const float *params) {
  if (!g || !params) {
    pdlp::g_last_error = "bad argument to pdlp_gnn_set_params";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    for (int64_t e = 0; e < pdlp::gnn::kNumParams; ++e)
      if (!std::isfinite(params[e])) pdlp::raise(PDLP_ERR_ARG, "non-finite parameter");
    HIPCHK(hipDeviceSynchronize());
    g->model.set_params(params, nullptr);
  });
}

int pdlp_gnn_set_omega_weight(pdlp_gnn *g, float w) {
  if (!g || !std::isfinite(w) || w < 0.f) {
    pdlp::g_last_error = "bad argument to pdlp_gnn_set_omega_weight";
    return PDLP_ERR_ARG;
  }
  g->model.omega_weight = w;
  return PDLP_OK;
}

int pdlp_gnn_predict(pdlp_gnn *g, pdlp_problem *p, double *x0, double *y0, double *omega0) {
  if (!g || !p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return with_graph(g, p->s, [&](const pdlp::gnn::GraphView &v) {
    gnn_predict(g->model, v, x0, y0, omega0, nullptr, nullptr, nullptr);
  });
}

int pdlp_gnn_predict_batch(pdlp_gnn *g, pdlp_batch *b, double *x0, double *y0, double *omega0) {
  if (!g || !b) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return with_graph(g, b->s, [&](const pdlp::gnn::GraphView &v) {
    gnn_predict(g->model, v, x0, y0, omega0, nullptr, nullptr, nullptr);
  });
}

int pdlp_gnn_predict_raw(pdlp_gnn *g, pdlp_batch *b, float *xhat, float *yhat, float *logw) {
  if (!g || !b) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return with_graph(g, b->s, [&](const pdlp::gnn::GraphView &v) {
    gnn_predict(g->model, v, nullptr, nullptr, nullptr, xhat, yhat, logw);
  });
}

int pdlp_gnn_gradients(pdlp_gnn *g, pdlp_batch *b, const double *x_star, const double *y_star,
                       const double *omega_star, double *loss, float *grad) {
  if (!g || !b || !x_star || !y_star || !omega_star) {
    pdlp::g_last_error = "bad argument to pdlp_gnn_gradients";
    return PDLP_ERR_ARG;
  }
  return with_graph(g, b->s, [&](const pdlp::gnn::GraphView &v) {
    auto &M = g->model;
    const float *av = nullptr, *tv = nullptr;
    M.prepare(v, av, tv, true);
    M.load_targets(v, x_star, y_star, omega_star);
    M.forward(v, av, tv, true);
    M.backward(v, av, tv);
    const double L = M.loss(v);
    if (loss) *loss = L;
    if (grad) HIPCHK(hipMemcpy(grad, M.G, sizeof(float) * pdlp::gnn::kNumParams, hipMemcpyDeviceToHost));
  });
}

int pdlp_gnn_train_step(pdlp_gnn *g, pdlp_batch *b, const double *x_star, const double *y_star,
                        const double *omega_star, float lr, double *loss) {
  if (!g || !b || !x_star || !y_star || !omega_star || !(lr > 0.f)) {
    pdlp::g_last_error = "bad argument to pdlp_gnn_train_step";
    return PDLP_ERR_ARG;
  }
  return with_graph(g, b->s, [&](const pdlp::gnn::GraphView &v) {
    using namespace pdlp::gnn;
    auto &M = g->model;
    const float *av = nullptr, *tv = nullptr;
    M.prepare(v, av, tv, true);
    M.load_targets(v, x_star, y_star, omega_star);
    M.forward(v, av, tv, true);
    M.backward(v, av, tv);
    M.step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)M.step), c2 = 1.f - std::pow(b2, (float)M.step);
    hipLaunchKernelGGL(g_adam, dim3(grid_cap(kNumParams, kGB, 1024)), dim3(kGB), 0, v.stream, (int32_t)kNumParams,
                       M.P, (const float *)M.G, M.M1, M.M2, lr, b1, b2, 1e-8f, c1, c2);
    HIPCHK(hipGetLastError());
    const double L = M.loss(v);
    if (loss) *loss = L;
  });
}

void pdlp_gnn_destroy(pdlp_gnn *g) {
  if (g) (void)hipDeviceSynchronize();
  delete g;
}

int pdlp_batch_get_scaling(pdlp_batch *b, double *Dr, double *Dc, double *scaled_val) {
  if (!b) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { b->s.visit([&](auto &s) { s.get_scaling(Dr, Dc, scaled_val); }); });
}

int pdlp_batch_get_internal(pdlp_batch *b, int32_t *row_ptr, int32_t *col, double *val, int32_t *t_row_ptr,
                            int32_t *t_col, double *t_val, int32_t *row_perm, int32_t *col_perm) {
  if (!b) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    b->s.visit([&](auto &s) { s.get_internal(row_ptr, col, val, t_row_ptr, t_col, t_val, row_perm, col_perm); });
  });
}

}  // extern "C"
