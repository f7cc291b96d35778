// Kernels of the learned warm start: a bipartite variable/constraint message-passing network with
// hidden width 64 that predicts the scaled primal x, dual y and log primal weight of each LP from
// its scaled data. Activations are FP32, [node][64] row-major. Every dense product runs on the
// gfx950 BF16 matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation) with both operands rounded
// to BF16 (nearest even) as they are loaded; sparse products, heads, pooling and the optimiser are
// FP32 vector code. All reductions run in a fixed order, so results are bitwise reproducible.
//
// MFMA 16x16x16 lane layout (lane l of 64, v = 0..3, r = 0..3):
//   A operand  (16 x 16, row i, depth k):  i = l % 16, k = 4 (l / 16) + v
//   B operand  (16 x 16, depth k, col j):  j = l % 16, k = 4 (l / 16) + v
//   D result   (16 x 16):                  register r holds row 4 (l / 16) + r, column l % 16
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdlp {
namespace gnn {

constexpr int kH = 64;       // hidden width
constexpr int kF = 8;        // input features per node
constexpr int kLayers = 3;   // message-passing rounds
constexpr int kGB = 256;     // threads per block
constexpr int kChunk = 1024; // nodes per head / pooling chunk

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ short bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ bf16x4 to_bf16x4(float a, float b, float c, float d) {
  bf16x4 r;
  r[0] = bf16_bits(a), r[1] = bf16_bits(b), r[2] = bf16_bits(c), r[3] = bf16_bits(d);
  return r;
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double slog(double v) { return v < 0.0 ? -log1p(-v) : log1p(v); }

// ------------------------------------------------------------------------------------------------
// Node features from the scaled problem (internal numbering).
//   variable j:   slog c, [l finite], [u finite], slog l (or 0), slog u (or 0), log(1 + deg)/4, 1, 0
//   constraint i: slog b, [<=], [>=], [=], log(1 + deg)/4, 1, 0, 0
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kGB) void g_features(int32_t m, int32_t n, const double *__restrict__ c,
                                                  const double *__restrict__ l, const double *__restrict__ u,
                                                  const int32_t *__restrict__ t_rp, const double *__restrict__ b,
                                                  const uint8_t *__restrict__ sense,
                                                  const int32_t *__restrict__ a_rp, float *__restrict__ fv,
                                                  float *__restrict__ fc) {
  const int32_t tot = m + n;
  for (int32_t t = blockIdx.x * kGB + threadIdx.x; t < tot; t += gridDim.x * kGB) {
    float f[kF];
    if (t < n) {
      const int32_t j = t;
      const bool lf = isfinite(l[j]), uf = isfinite(u[j]);
      f[0] = (float)slog(c[j]);
      f[1] = lf ? 1.f : 0.f;
      f[2] = uf ? 1.f : 0.f;
      f[3] = lf ? (float)slog(l[j]) : 0.f;
      f[4] = uf ? (float)slog(u[j]) : 0.f;
      f[5] = (float)(log1p((double)(t_rp[j + 1] - t_rp[j])) / 4.0);
      f[6] = 1.f;
      f[7] = 0.f;
      float4 *o = reinterpret_cast<float4 *>(fv + (int64_t)j * kF);
      o[0] = make_float4(f[0], f[1], f[2], f[3]);
      o[1] = make_float4(f[4], f[5], f[6], f[7]);
    } else {
      const int32_t i = t - n;
      const uint8_t s = sense[i];
      f[0] = (float)slog(b[i]);
      f[1] = s == 'L' ? 1.f : 0.f;
      f[2] = s == 'G' ? 1.f : 0.f;
      f[3] = s == 'E' ? 1.f : 0.f;
      f[4] = (float)(log1p((double)(a_rp[i + 1] - a_rp[i])) / 4.0);
      f[5] = 1.f;
      f[6] = 0.f;
      f[7] = 0.f;
      float4 *o = reinterpret_cast<float4 *>(fc + (int64_t)i * kF);
      o[0] = make_float4(f[0], f[1], f[2], f[3]);
      o[1] = make_float4(f[4], f[5], f[6], f[7]);
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Dense layer, forward:  out = relu(X1 W1 + X2 W2 + bias)   (X2 W2 only when TWO)
// X1 [R x K1] (K1 = 8 or 64), X2 [R x 64], W1 [K1 x 64], W2 [64 x 64] row-major FP32.
// One wave computes 16-row tiles (grid-stride), weights held in registers as BF16 fragments.
// ------------------------------------------------------------------------------------------------
template <int K1>
__device__ __forceinline__ void load_w_frags(const float *__restrict__ W, bf16x4 (&f)[(K1 + 15) / 16][4], int lane) {
  // B[k][j] = W[k][j]: lane holds k = 16 s + 4 (lane / 16) + v, j = 16 cb + lane % 16
#pragma unroll
  for (int s = 0; s < (K1 + 15) / 16; ++s)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      float t[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 16 * s + 4 * (lane / 16) + v;
        t[v] = k < K1 ? W[k * kH + 16 * cb + lane % 16] : 0.f;
      }
      f[s][cb] = to_bf16x4(t[0], t[1], t[2], t[3]);
    }
}

// A fragment of rows [row0, row0 + 16) of X [R x K] at depth step s: row row0 + lane % 16,
// columns 16 s + 4 (lane / 16) + 0..3 (zero outside the matrix)
template <int K>
__device__ __forceinline__ bf16x4 load_a_rowmajor(const float *__restrict__ X, int32_t R, int32_t row0, int s, int lane) {
  const int32_t row = row0 + lane % 16;
  const int k = 16 * s + 4 * (lane / 16);
  if (row >= R || k >= K) return to_bf16x4(0.f, 0.f, 0.f, 0.f);
  const float4 v = *reinterpret_cast<const float4 *>(X + (int64_t)row * K + k);
  return to_bf16x4(v.x, v.y, v.z, v.w);
}

template <int K1, bool TWO>
__global__ __launch_bounds__(kGB) void g_dense_fwd(int32_t R, const float *__restrict__ X1, const float *__restrict__ W1,
                                                   const float *__restrict__ X2, const float *__restrict__ W2,
                                                   const float *__restrict__ bias, float *__restrict__ out) {
  constexpr int S1 = (K1 + 15) / 16;
  const int lane = threadIdx.x % 64;
  const int wave = blockIdx.x * (kGB / 64) + threadIdx.x / 64;
  const int nwaves = gridDim.x * (kGB / 64);
  bf16x4 w1[S1][4];
  load_w_frags<K1>(W1, w1, lane);
  bf16x4 w2[4][4];
  if (TWO) load_w_frags<kH>(W2, w2, lane);
  float bj[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) bj[cb] = bias[16 * cb + lane % 16];
  const int32_t ntiles = (R + 15) / 16;
  for (int32_t tile = wave; tile < ntiles; tile += nwaves) {
    const int32_t row0 = tile * 16;
    f32x4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const bf16x4 a = load_a_rowmajor<K1>(X1, R, row0, s, lane);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma16(a, w1[s][cb], acc[cb]);
    }
    if (TWO) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bf16x4 a = load_a_rowmajor<kH>(X2, R, row0, s, lane);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma16(a, w2[s][cb], acc[cb]);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int32_t row = row0 + 4 * (lane / 16) + r;
      if (row < R) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) out[(int64_t)row * kH + 16 * cb + lane % 16] = fmaxf(acc[cb][r] + bj[cb], 0.f);
      }
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Dense layer, backward. With P = dout * [out > 0] (the pre-activation gradient):
//   dX1 = P W1'   (when DX1),   dX2 = P W2'   (when TWO),
//   per-wave partial sums of  dW1 = X1' P,  dW2 = X2' P,  db = column sums of P,
// written to part[wave][K1*64 (+ 4096) + 64] for g_reduce_waves.
// ------------------------------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void load_wt_frags(const float *__restrict__ W, bf16x4 (&f)[4][(K + 15) / 16], int lane) {
  // B[k][c] = W[c][k] (W is [K x 64]); lane holds k = 16 s + 4 (lane / 16) + v, c = 16 cb + lane % 16
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int cb = 0; cb < (K + 15) / 16; ++cb) {
      const int c = 16 * cb + lane % 16;
      const int k = 16 * s + 4 * (lane / 16);
      if (c < K) {
        const float4 v = *reinterpret_cast<const float4 *>(W + c * kH + k);
        f[s][cb] = to_bf16x4(v.x, v.y, v.z, v.w);
      } else {
        f[s][cb] = to_bf16x4(0.f, 0.f, 0.f, 0.f);
      }
    }
}

// A fragment of X' (channels x nodes) for the weight gradient: channel 16 ib + lane % 16,
// nodes row0 + 4 (lane / 16) + v
template <int K>
__device__ __forceinline__ bf16x4 load_a_transposed(const float *__restrict__ X, int32_t R, int32_t row0, int ib,
                                                    int lane) {
  const int c = 16 * ib + lane % 16;
  float t[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int32_t row = row0 + 4 * (lane / 16) + v;
    t[v] = (c < K && row < R) ? X[(int64_t)row * K + c] : 0.f;
  }
  return to_bf16x4(t[0], t[1], t[2], t[3]);
}

template <int K1, bool TWO, bool DX1>
__global__ __launch_bounds__(kGB) void g_dense_bwd(int32_t R, const float *__restrict__ out,
                                                   const float *__restrict__ dout, const float *__restrict__ X1,
                                                   const float *__restrict__ W1, const float *__restrict__ X2,
                                                   const float *__restrict__ W2, float *__restrict__ dX1,
                                                   float *__restrict__ dX2, float *__restrict__ part) {
  constexpr int IB1 = (K1 + 15) / 16;
  constexpr int LEN = K1 * kH + (TWO ? kH * kH : 0) + kH;
  const int lane = threadIdx.x % 64;
  const int wave = blockIdx.x * (kGB / 64) + threadIdx.x / 64;
  const int nwaves = gridDim.x * (kGB / 64);
  bf16x4 w1t[4][IB1], w2t[4][4];
  if (DX1) load_wt_frags<K1>(W1, w1t, lane);
  if (TWO) load_wt_frags<kH>(W2, w2t, lane);
  f32x4 gw1[IB1][4], gw2[4][4];
#pragma unroll
  for (int ib = 0; ib < IB1; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) gw1[ib][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) gw2[ib][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
  float gb[4] = {0.f, 0.f, 0.f, 0.f};

  const int32_t ntiles = (R + 15) / 16;
  for (int32_t tile = wave; tile < ntiles; tile += nwaves) {
    const int32_t row0 = tile * 16;
    // P in the D layout (nodes 4 (lane/16) + r, channel 16 jb + lane % 16): B operand of X' P
    bf16x4 pD[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      float t[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int32_t row = row0 + 4 * (lane / 16) + r;
        const int64_t o = (int64_t)row * kH + 16 * jb + lane % 16;
        t[r] = (row < R && out[o] > 0.f) ? dout[o] : 0.f;
        gb[jb] += t[r];
      }
      pD[jb] = to_bf16x4(t[0], t[1], t[2], t[3]);
    }
#pragma unroll
    for (int ib = 0; ib < IB1; ++ib) {
      const bf16x4 a = load_a_transposed<K1>(X1, R, row0, ib, lane);
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) gw1[ib][jb] = mfma16(a, pD[jb], gw1[ib][jb]);
    }
    if (TWO) {
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) {
        const bf16x4 a = load_a_transposed<kH>(X2, R, row0, ib, lane);
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) gw2[ib][jb] = mfma16(a, pD[jb], gw2[ib][jb]);
      }
    }
    if (DX1 || TWO) {
      // P in the A layout (node row0 + lane % 16, channels 16 s + 4 (lane / 16) + v)
      bf16x4 pA[4];
      const int32_t rowA = row0 + lane % 16;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 16 * s + 4 * (lane / 16);
        if (rowA < R) {
          const float4 o = *reinterpret_cast<const float4 *>(out + (int64_t)rowA * kH + k);
          const float4 g = *reinterpret_cast<const float4 *>(dout + (int64_t)rowA * kH + k);
          pA[s] = to_bf16x4(o.x > 0.f ? g.x : 0.f, o.y > 0.f ? g.y : 0.f, o.z > 0.f ? g.z : 0.f,
                            o.w > 0.f ? g.w : 0.f);
        } else {
          pA[s] = to_bf16x4(0.f, 0.f, 0.f, 0.f);
        }
      }
      if (DX1) {
#pragma unroll
        for (int cb = 0; cb < IB1; ++cb) {
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < 4; ++s) acc = mfma16(pA[s], w1t[s][cb], acc);
          const int c = 16 * cb + lane % 16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int32_t row = row0 + 4 * (lane / 16) + r;
            if (row < R && c < K1) dX1[(int64_t)row * K1 + c] = acc[r];
          }
        }
      }
      if (TWO) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < 4; ++s) acc = mfma16(pA[s], w2t[s][cb], acc);
          const int c = 16 * cb + lane % 16;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int32_t row = row0 + 4 * (lane / 16) + r;
            if (row < R) dX2[(int64_t)row * kH + c] = acc[r];
          }
        }
      }
    }
  }
  // per-wave partials: dW rows c = 16 ib + 4 (lane / 16) + r, columns j = 16 jb + lane % 16
  float *pw = part + (int64_t)wave * LEN;
#pragma unroll
  for (int ib = 0; ib < IB1; ++ib)
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 16 * ib + 4 * (lane / 16) + r;
        if (c < K1) pw[c * kH + 16 * jb + lane % 16] = gw1[ib][jb][r];
      }
  if (TWO) {
    float *pw2 = pw + K1 * kH;
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) pw2[(16 * ib + 4 * (lane / 16) + r) * kH + 16 * jb + lane % 16] = gw2[ib][jb][r];
  }
  // bias: lanes l, l^16, l^32, l^48 hold the same channel
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) {
    float v = gb[jb];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < 16) pw[LEN - kH + 16 * jb + lane] = v;
  }
}

// grad[e] = sum over waves w (in order) of part[w][e], e < len
__global__ __launch_bounds__(kGB) void g_reduce_waves(int32_t nw, int32_t len, const float *__restrict__ part,
                                                      float *__restrict__ grad) {
  for (int32_t e = blockIdx.x * kGB + threadIdx.x; e < len; e += gridDim.x * kGB) {
    double s = 0.0;
    for (int32_t w = 0; w < nw; ++w) s += (double)part[(int64_t)w * len + e];
    grad[e] = (float)s;
  }
}

// ------------------------------------------------------------------------------------------------
// Sparse product with 64-channel rows:  out[r] = (ACC ? out[r] : 0) + sum_e val[e] in[ci[e]]
// 16 lanes per row, 4 channels (one float4) per lane; FP32 accumulation in nonzero order.
// ------------------------------------------------------------------------------------------------
template <bool ACC>
__global__ __launch_bounds__(kGB) void g_spmm(int32_t R, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                              const float *__restrict__ val, const float *__restrict__ in,
                                              float *__restrict__ out) {
  const int q = threadIdx.x % 16;
  for (int32_t r = blockIdx.x * (kGB / 16) + threadIdx.x / 16; r < R; r += gridDim.x * (kGB / 16)) {
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    const int32_t e1 = rp[r + 1];
    int32_t e = rp[r];
    for (; e + 1 < e1; e += 2) {
      const int32_t c0 = ci[e], c1 = ci[e + 1];
      const float v0 = val[e], v1 = val[e + 1];
      const float4 x0 = *reinterpret_cast<const float4 *>(in + (int64_t)c0 * kH + 4 * q);
      const float4 x1 = *reinterpret_cast<const float4 *>(in + (int64_t)c1 * kH + 4 * q);
      s.x += v0 * x0.x, s.y += v0 * x0.y, s.z += v0 * x0.z, s.w += v0 * x0.w;
      s.x += v1 * x1.x, s.y += v1 * x1.y, s.z += v1 * x1.z, s.w += v1 * x1.w;
    }
    if (e < e1) {
      const float v0 = val[e];
      const float4 x0 = *reinterpret_cast<const float4 *>(in + (int64_t)ci[e] * kH + 4 * q);
      s.x += v0 * x0.x, s.y += v0 * x0.y, s.z += v0 * x0.z, s.w += v0 * x0.w;
    }
    float4 *o = reinterpret_cast<float4 *>(out + (int64_t)r * kH + 4 * q);
    if (ACC) {
      const float4 t = *o;
      s.x += t.x, s.y += t.y, s.z += t.z, s.w += t.w;
    }
    *o = s;
  }
}

// ------------------------------------------------------------------------------------------------
// Heads, pooling and loss. Nodes of one side are cut into chunks (cs[k], ce[k]) of one instance
// cq[k] each; a block handles one chunk. 16 lanes per node, 4 channels per lane.
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ float dot16(float4 h, float4 w) {
  float d = h.x * w.x + h.y * w.y + h.z * w.z + h.w * w.w;
  d += __shfl_xor(d, 1);
  d += __shfl_xor(d, 2);
  d += __shfl_xor(d, 4);
  d += __shfl_xor(d, 8);
  return d;
}

// pred = h w + b0; pool[k] = sum of h rows over the chunk; if tgt: sq[k] = sum (pred - tgt)^2
__global__ __launch_bounds__(kGB) void g_head_fwd(const int32_t *__restrict__ cs, const int32_t *__restrict__ ce,
                                                  const float *__restrict__ h, const float *__restrict__ w,
                                                  const float *__restrict__ b0, const float *__restrict__ tgt,
                                                  float *__restrict__ pred, float *__restrict__ pool,
                                                  double *__restrict__ sq) {
  __shared__ float4 red[kGB];
  __shared__ double rsq[kGB / 16];
  const int k = blockIdx.x, q = threadIdx.x % 16, slot = threadIdx.x / 16;
  const float4 wq = make_float4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
  const float bias = b0[0];
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  double e2 = 0.0;
  for (int32_t j = cs[k] + slot; j < ce[k]; j += kGB / 16) {
    const float4 hv = *reinterpret_cast<const float4 *>(h + (int64_t)j * kH + 4 * q);
    acc.x += hv.x, acc.y += hv.y, acc.z += hv.z, acc.w += hv.w;
    const float p = dot16(hv, wq) + bias;
    if (q == 0) {
      pred[j] = p;
      if (tgt) {
        const double d = (double)p - (double)tgt[j];
        e2 += d * d;
      }
    }
  }
  red[threadIdx.x] = acc;
  if (q == 0) rsq[slot] = e2;
  __syncthreads();
  if (threadIdx.x < 16) {
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int t = 0; t < kGB / 16; ++t) {
      const float4 v = red[t * 16 + threadIdx.x];
      s.x += v.x, s.y += v.y, s.z += v.z, s.w += v.w;
    }
    *reinterpret_cast<float4 *>(pool + (int64_t)k * kH + 4 * threadIdx.x) = s;
  }
  if (threadIdx.x == 0 && sq) {
    double s = 0.0;
    for (int t = 0; t < kGB / 16; ++t) s += rsq[t];
    sq[k] = s;
  }
}

// Per instance q (one block of 64 threads): pooled means, log omega, loss terms and dL/dlog omega.
//   pv, pc [K x 64]; logw [K]; if tw: lossq[q] = sqx/n_q + sqy/m_q + w_om (logw - tw)^2,
//   dlw = 2 w_om (logw - tw)/K
__global__ __launch_bounds__(64) void g_head_inst(int32_t K, const int32_t *__restrict__ col0,
                                                  const int32_t *__restrict__ row0,
                                                  const int32_t *__restrict__ vch0, const int32_t *__restrict__ cch0,
                                                  const float *__restrict__ vpool, const float *__restrict__ cpool,
                                                  const double *__restrict__ vsq, const double *__restrict__ csq,
                                                  const float *__restrict__ wov, const float *__restrict__ woc,
                                                  const float *__restrict__ bo, const float *__restrict__ tw,
                                                  float w_om, float *__restrict__ pv, float *__restrict__ pc,
                                                  float *__restrict__ logw, double *__restrict__ lossq,
                                                  float *__restrict__ dlw) {
  __shared__ float red[64];
  const int q = blockIdx.x, ch = threadIdx.x;
  const int32_t nq = col0[q + 1] - col0[q], mq = row0[q + 1] - row0[q];
  float sv = 0.f, sc = 0.f;
  for (int32_t k = vch0[q]; k < vch0[q + 1]; ++k) sv += vpool[(int64_t)k * kH + ch];
  for (int32_t k = cch0[q]; k < cch0[q + 1]; ++k) sc += cpool[(int64_t)k * kH + ch];
  sv /= (float)max(nq, 1);
  sc /= (float)max(mq, 1);
  pv[(int64_t)q * kH + ch] = sv;
  pc[(int64_t)q * kH + ch] = sc;
  red[ch] = sv * wov[ch] + sc * woc[ch];
  __syncthreads();
  if (ch == 0) {
    float s = 0.f;
    for (int t = 0; t < 64; ++t) s += red[t];
    const float lw = s + bo[0];
    logw[q] = lw;
    if (tw) {
      double sx = 0.0, sy = 0.0;
      for (int32_t k = vch0[q]; k < vch0[q + 1]; ++k) sx += vsq[k];
      for (int32_t k = cch0[q]; k < cch0[q + 1]; ++k) sy += csq[k];
      const double d = (double)lw - (double)tw[q];
      lossq[q] = (nq ? sx / nq : 0.0) + (mq ? sy / mq : 0.0) + (double)w_om * d * d;
      dlw[q] = (float)(2.0 * (double)w_om * d / K);
    }
  }
}

// Head backward for one side: d = 2 (pred - tgt) / (size_q K) per node,
//   dh[j] = d w + (dlw[q] / size_q) wo                  (gradient entering the top layer)
//   gpart[k] = [sum_j d h[j] (64), sum_j d]             (per chunk)
__global__ __launch_bounds__(kGB) void g_head_bwd(int32_t K, const int32_t *__restrict__ cs,
                                                  const int32_t *__restrict__ ce, const int32_t *__restrict__ cq,
                                                  const int32_t *__restrict__ off0, const float *__restrict__ h,
                                                  const float *__restrict__ pred, const float *__restrict__ tgt,
                                                  const float *__restrict__ w, const float *__restrict__ wo,
                                                  const float *__restrict__ dlw, float *__restrict__ dh,
                                                  float *__restrict__ gpart) {
  __shared__ float4 red[kGB];
  __shared__ float rb[kGB / 16];
  const int k = blockIdx.x, q = threadIdx.x % 16, slot = threadIdx.x / 16;
  const int32_t inst = cq[k];
  const int32_t sz = max(off0[inst + 1] - off0[inst], 1);
  // head vectors sit at odd offsets of the parameter vector: scalar loads
  const float4 wq = make_float4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
  const float4 woq = make_float4(wo[4 * q], wo[4 * q + 1], wo[4 * q + 2], wo[4 * q + 3]);
  const float pool_g = dlw[inst] / (float)sz;
  const float scale = 2.0f / ((float)sz * (float)K);
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  float accb = 0.f;
  for (int32_t j = cs[k] + slot; j < ce[k]; j += kGB / 16) {
    const float d = (pred[j] - tgt[j]) * scale;
    const float4 hv = *reinterpret_cast<const float4 *>(h + (int64_t)j * kH + 4 * q);
    acc.x += d * hv.x, acc.y += d * hv.y, acc.z += d * hv.z, acc.w += d * hv.w;
    accb += d;
    float4 g;
    g.x = d * wq.x + pool_g * woq.x, g.y = d * wq.y + pool_g * woq.y;
    g.z = d * wq.z + pool_g * woq.z, g.w = d * wq.w + pool_g * woq.w;
    *reinterpret_cast<float4 *>(dh + (int64_t)j * kH + 4 * q) = g;
  }
  red[threadIdx.x] = acc;
  if (q == 0) rb[slot] = accb;
  __syncthreads();
  if (threadIdx.x < 16) {
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int t = 0; t < kGB / 16; ++t) {
      const float4 v = red[t * 16 + threadIdx.x];
      s.x += v.x, s.y += v.y, s.z += v.z, s.w += v.w;
    }
    *reinterpret_cast<float4 *>(gpart + (int64_t)k * (kH + 1) + 4 * threadIdx.x) = s;
  }
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int t = 0; t < kGB / 16; ++t) s += rb[t];
    gpart[(int64_t)k * (kH + 1) + kH] = s;
  }
}

// Head parameter gradients (one block of 64 threads):
//   gw (64) + gb (1) = sum over chunks of gpart;  gwo (64) = sum_q pooled[q] dlw[q];  gbo = sum_q dlw[q]
__global__ __launch_bounds__(64) void g_head_fin(int32_t nch, const float *__restrict__ gpart, int32_t K,
                                                 const float *__restrict__ pooled, const float *__restrict__ dlw,
                                                 float *__restrict__ gw, float *__restrict__ gb,
                                                 float *__restrict__ gwo, float *__restrict__ gbo) {
  const int ch = threadIdx.x;
  double s = 0.0, so = 0.0;
  for (int32_t k = 0; k < nch; ++k) s += (double)gpart[(int64_t)k * (kH + 1) + ch];
  for (int32_t q = 0; q < K; ++q) so += (double)pooled[(int64_t)q * kH + ch] * (double)dlw[q];
  gw[ch] = (float)s;
  gwo[ch] = (float)so;
  if (ch == 0) {
    double sb = 0.0, sbo = 0.0;
    for (int32_t k = 0; k < nch; ++k) sb += (double)gpart[(int64_t)k * (kH + 1) + kH];
    for (int32_t q = 0; q < K; ++q) sbo += (double)dlw[q];
    gb[0] = (float)sb;
    if (gbo) gbo[0] = (float)sbo;
  }
}

// ------------------------------------------------------------------------------------------------
// Adam on the FP32 master weights (bias-corrected moments).
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kGB) void g_adam(int32_t np, float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m1, float *__restrict__ m2, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
  for (int32_t e = blockIdx.x * kGB + threadIdx.x; e < np; e += gridDim.x * kGB) {
    const float ge = g[e];
    const float a = b1 * m1[e] + (1.f - b1) * ge;
    const float b = b2 * m2[e] + (1.f - b2) * ge * ge;
    m1[e] = a, m2[e] = b;
    p[e] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
  }
}

// ------------------------------------------------------------------------------------------------
// Numbering and scaling at the boundary.
// ------------------------------------------------------------------------------------------------
// targets, scaled and in internal numbering: t[j] = ext[perm[j]] / D[j]
__global__ __launch_bounds__(kGB) void g_target(int32_t n, const double *__restrict__ ext,
                                                const int32_t *__restrict__ perm, const double *__restrict__ D,
                                                float *__restrict__ t) {
  for (int32_t j = blockIdx.x * kGB + threadIdx.x; j < n; j += gridDim.x * kGB) t[j] = (float)(ext[perm[j]] / D[j]);
}
// predictions in the caller's numbering and the original space: ext[e] = D[inv[e]] pred[inv[e]]
__global__ __launch_bounds__(kGB) void g_unscale_pred(int32_t n, const float *__restrict__ pred,
                                                      const int32_t *__restrict__ inv, const double *__restrict__ D,
                                                      double *__restrict__ ext) {
  for (int32_t e = blockIdx.x * kGB + threadIdx.x; e < n; e += gridDim.x * kGB) {
    const int32_t j = inv[e];
    ext[e] = D[j] * (double)pred[j];
  }
}
__global__ __launch_bounds__(kGB) void g_to_float(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
  for (int64_t e = blockIdx.x * (int64_t)kGB + threadIdx.x; e < n; e += (int64_t)gridDim.x * kGB) b[e] = (float)a[e];
}

}  // namespace gnn
}  // namespace pdlp
