// HIP kernels of libpdlp for gfx950 (CDNA4, wave64).
//
// Iteration kernels (one PDHG attempt = k_dual, k_step, k_primal; every eval_every attempts k_eval,
// k_eval_fin, k_restart), set-up kernels (transpose, scan, scaling) and finalize kernels. All
// reductions are deterministic: fixed per-thread order, fixed wave/block trees, block partials
// summed in block order by a one-block-per-instance kernel launched after the producer (the kernel
// boundary orders the partial sums; no block issues a device-scope fence).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pdlp_internal.h"

namespace pdlp {

// ----------------------------------------------------------------------------------------------
// Small device helpers
// ----------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T clipv(T x, T lo, T hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

// Projection onto the dual sign set of a row: 'G' -> [0, inf), 'L' -> (-inf, 0], 'E' -> R.
template <typename T>
__device__ __forceinline__ T proj_dual(T y, uint8_t s) {
  if (s == 'G') return y > T(0) ? y : T(0);
  if (s == 'L') return y < T(0) ? y : T(0);
  return y;
}

// Primal residual of a row given b - a'x.
__device__ __forceinline__ double row_violation(double t, uint8_t s) {
  if (s == 'G') return t > 0.0 ? t : 0.0;
  if (s == 'L') return t < 0.0 ? t : 0.0;
  return t;
}

// Projection of g onto the reduced-cost set fixed by which bounds are finite.
__device__ __forceinline__ double proj_reduced(double g, double lo, double hi) {
  const bool lf = isfinite(lo), uf = isfinite(hi);
  if (lf && uf) return g;
  if (lf) return g > 0.0 ? g : 0.0;
  if (uf) return g < 0.0 ? g : 0.0;
  return 0.0;
}

// Contribution of one column to the dual objective: l lambda^+ - u lambda^-.
__device__ __forceinline__ double bound_term(double lo, double hi, double lam) {
  double t = 0.0;
  if (isfinite(lo) && lam > 0.0) t += lo * lam;
  if (isfinite(hi) && lam < 0.0) t += hi * lam;
  return t;
}

template <typename A>
__device__ __forceinline__ A wave_sum(A v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide sum of NV doubles; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double red[NV * kWaves];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q * kWaves + wid] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = red[q * kWaves];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) s += red[q * kWaves + w];
      v[q] = s;
    }
  }
}

template <typename A>
__device__ __forceinline__ A block_sum_scalar(A v) {
  __shared__ A red1[kWaves];
  v = wave_sum(v);
  const int wid = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  __syncthreads();
  if (lane == 0) red1[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    A s = red1[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += red1[w];
    v = s;
  }
  return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs. Give every XCD a contiguous range of an
// instance's work blocks so that neighbouring chunks (which gather neighbouring parts of x in
// structured matrices) share that XCD's L2.
__host__ __device__ __forceinline__ int xcd_remap(int bid, int nb) {
  constexpr int kXcd = 8;
  if (nb < kXcd) return bid;
  const int xcd = bid % kXcd, local = bid / kXcd;
  const int base = nb / kXcd, extra = nb % kXcd;
  return xcd * base + (xcd < extra ? xcd : extra) + local;
}

// ----------------------------------------------------------------------------------------------
// Row-class chunk SpMV engine.
//
// Inside a handle the rows of A (and of A') are stored sorted by length class: class c holds the
// rows with 2^(c+1) <= len < 2^(c+2) (class 0: len <= 3, class 6: len >= 128), and a row of class
// c is summed by G = 2^c lanes. A chunk is a run of consecutive rows of one class holding a bounded
// number of nonzeros. A wave walks its chunks: lane groups of G take consecutive rows (so the 64
// lanes of a wave read one contiguous stretch of val/col even for the shortest rows), each lane
// sums its strided share with four independent accumulators (four loads and gathers in flight per
// lane), a G-lane shuffle tree finishes the row, and the group's first lane runs the row's
// epilogue epi(row, sum, prefetched operands).
// A chunk that is one row of at least kCoopNnz nonzeros is summed by the whole block (all four
// waves, LDS across waves) instead of one wave, so a few very long rows (the shared capacity
// columns of the energy models, the heavy tail of power-law rows) do not serialise on one wave.
// The summation order of a row depends only on its length, so results are deterministic.
// ----------------------------------------------------------------------------------------------
struct NoPre {};

// The two accumulation forms of the engine, spelled out so that every path that sums a row rounds
// identically: a rounded product and a rounded add (the library is built without floating-point
// contraction, so no product is fused into a sum), and for the masked slots a select against zero
// in between. The iteration products accumulate in FP64 in both precisions: an FP32 value times an
// FP32 value is exact in FP64, so an FP32 row sum carries only the rounding of its FP64 additions
// until it is stored.
template <typename Acc>
__device__ __forceinline__ Acc acc_fma(Acc s, Acc v, Acc x) {
  const Acc prod = v * x;
  return s + prod;
}
template <typename Acc>
__device__ __forceinline__ Acc acc_masked(Acc s, bool p, Acc v, Acc x) {
#pragma clang fp contract(off)
  const Acc prod = v * x;
  return s + (p ? prod : Acc(0));
}

template <typename V, typename X, typename Acc, typename Pre, typename Epi>
__device__ __forceinline__ void chunk_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                           const V *__restrict__ val, const X *__restrict__ x, int r0, int r1,
                                           int cls, Pre &&pre, Epi &&epi) {
  const int lane = (int)threadIdx.x & (kWave - 1);
  const int G = 1 << cls;
  const int grp = lane >> cls, gl = lane & (G - 1);
  const int per = kWave >> cls;
  using PF = decltype(pre(r0));
  for (int rb = r0; rb < r1; rb += per) {
    const int r = rb + grp;
    const bool act = r < r1;
    const PF pf = (act && gl == 0) ? pre(r) : PF{};
    Acc s0 = Acc(0), s1 = Acc(0), s2 = Acc(0), s3 = Acc(0);
    if (act) {
      const int k1 = rp[r + 1];
      // classes 0..5 give every lane at most four elements: one round of predicated loads, all
      // issued before the first use; class 6 loops. val/col are streamed once per product and
      // bypass the caches (non-temporal) so that x stays resident for the gathers.
      for (int e = rp[r] + gl; e < k1; e += 4 * G) {
        // branch-free: out-of-row slots re-read the row's last element and are masked out
        const bool p1 = e + G < k1, p2 = e + 2 * G < k1, p3 = e + 3 * G < k1;
        const int e1 = p1 ? e + G : k1 - 1, e2 = p2 ? e + 2 * G : k1 - 1, e3 = p3 ? e + 3 * G : k1 - 1;
        const int c0 = __builtin_nontemporal_load(ci + e), c1 = __builtin_nontemporal_load(ci + e1);
        const int c2 = __builtin_nontemporal_load(ci + e2), c3 = __builtin_nontemporal_load(ci + e3);
        const V v0 = __builtin_nontemporal_load(val + e), v1 = __builtin_nontemporal_load(val + e1);
        const V v2 = __builtin_nontemporal_load(val + e2), v3 = __builtin_nontemporal_load(val + e3);
        const X x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
        s0 = acc_fma(s0, Acc(v0), Acc(x0));
        s1 = acc_masked(s1, p1, Acc(v1), Acc(x1));
        s2 = acc_masked(s2, p2, Acc(v2), Acc(x2));
        s3 = acc_masked(s3, p3, Acc(v3), Acc(x3));
      }
    }
    Acc s = (s0 + s1) + (s2 + s3);
    for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (act && gl == 0) epi(r, s, pf);
  }
}

constexpr int kCoopNnz = 1024;
static_assert(kBlock == 4 * kWave, "coop_row maps the four accumulators of a lane onto four waves");

// Row r summed by all kBlock threads of the block with exactly the arithmetic of one wave of 64
// lanes (class 6): wave w computes the lanes' accumulator w (elements rp[r] + lane + 64 w + 256 i),
// the four accumulators meet in LDS, and wave 0 finishes with the same shuffle tree. The row sum is
// therefore bitwise the one chunk_rows gives; only the work is spread over four waves. Every thread
// of the block must call this (it contains block barriers); thread 0 runs the epilogue.
template <typename V, typename X, typename Acc, typename Pre, typename Epi>
__device__ __forceinline__ void coop_row(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                         const V *__restrict__ val, const X *__restrict__ x, int r, Acc *red,
                                         Pre &&pre, Epi &&epi) {
  const int tid = (int)threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  using PF = decltype(pre(r));
  const PF pf = tid == 0 ? pre(r) : PF{};
  const int k1 = rp[r + 1];
  Acc s = Acc(0);
  if (w == 0) {
    for (int e = rp[r] + lane; e < k1; e += 4 * kWave) {
      const int c0 = __builtin_nontemporal_load(ci + e);
      const V v0 = __builtin_nontemporal_load(val + e);
      s = acc_fma(s, Acc(v0), Acc(x[c0]));
    }
  } else {
    for (int e = rp[r] + lane; e < k1; e += 4 * kWave) {
      const bool p = e + w * kWave < k1;
      const int ew = p ? e + w * kWave : k1 - 1;
      const int c = __builtin_nontemporal_load(ci + ew);
      const V v = __builtin_nontemporal_load(val + ew);
      s = acc_masked(s, p, Acc(v), Acc(x[c]));
    }
  }
  red[tid] = s;
  __syncthreads();
  if (w == 0) {
    Acc t = (red[lane] + red[kWave + lane]) + (red[2 * kWave + lane] + red[3 * kWave + lane]);
    for (int off = kWave >> 1; off > 0; off >>= 1) t += __shfl_xor(t, off, kWave);
    if (lane == 0) epi(r, t, pf);
  }
  __syncthreads();
}

__device__ __forceinline__ bool long_chunk(const int32_t *__restrict__ rp, const int32_t *__restrict__ chunk_row,
                                           const int8_t *__restrict__ chunk_cls, int c) {
  if (chunk_cls[c] != 6) return false;
  const int r = chunk_row[c];
  return chunk_row[c + 1] == r + 1 && rp[r + 1] - rp[r] >= kCoopNnz;
}

// The chunks [c_lo, c_hi) of a block: runs of ordinary chunks are shared out over the waves (wave w
// takes the run's chunks w, w + 4, ...); a long single-row chunk is summed by the whole block. The
// range is the same for every thread of the block, so all of them meet the same barriers.
template <typename V, typename X, typename Acc, typename Pre, typename Epi>
__device__ __forceinline__ void block_chunks(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                             const V *__restrict__ val, const X *__restrict__ x,
                                             const int32_t *__restrict__ chunk_row,
                                             const int8_t *__restrict__ chunk_cls, int c_lo, int c_hi, Pre &&pre,
                                             Epi &&epi) {
  __shared__ Acc red[kBlock];
  const int wave = (int)threadIdx.x >> 6;
  int ch = c_lo;
  while (ch < c_hi) {
    int stop = ch;
    while (stop < c_hi && !long_chunk(rp, chunk_row, chunk_cls, stop)) ++stop;
    for (int c = ch + wave; c < stop; c += kWaves)
      chunk_rows<V, X, Acc>(rp, ci, val, x, chunk_row[c], chunk_row[c + 1], chunk_cls[c], pre, epi);
    if (stop < c_hi) {
      coop_row<V, X, Acc>(rp, ci, val, x, chunk_row[stop], red, pre, epi);
      ++stop;
    }
    ch = stop;
  }
}

// Sum of per-block partials [b0, b1) x [NV] in a fixed order; valid in thread 0.
template <int NV>
__device__ __forceinline__ void final_sum(const double *partials, int b0, int b1, double (&out)[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) out[q] = 0.0;
  for (int bidx = b0 + (int)threadIdx.x; bidx < b1; bidx += kBlock) {
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] += partials[(size_t)bidx * NV + q];
  }
  block_sum<NV>(out);
}

__device__ __forceinline__ void mark_done(State *st, int32_t *ndone) {
  if (!st->done) {
    st->done = 1;
    atomicAdd(ndone, 1);
  }
}

// A work block of an instance: which instance, its index among the instance's blocks (remapped
// so that each XCD owns a contiguous range) and how many blocks the instance has.
struct WBlock {
  int inst, lb, nb;
};
__device__ __forceinline__ WBlock work_block(const int32_t *__restrict__ b0, const int32_t *__restrict__ binst) {
  WBlock w;
  w.inst = binst[blockIdx.x];
  const int s = b0[w.inst];
  w.nb = b0[w.inst + 1] - s;
  w.lb = xcd_remap((int)blockIdx.x - s, w.nb);
  return w;
}
// y = A x over every instance's chunks (plain store epilogue); grid: the work blocks of the side.
template <typename V, typename X, typename Acc, typename Y>
__global__ __launch_bounds__(kBlock) void k_spmv(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                 const V *__restrict__ val, const int32_t *__restrict__ chunk_row,
                                                 const int8_t *__restrict__ chunk_cls, const int32_t *__restrict__ b0,
                                                 const int32_t *__restrict__ binst,
                                                 const int32_t *__restrict__ bchunk, const X *__restrict__ x,
                                                 Y *__restrict__ y) {
  const WBlock w = work_block(b0, binst);
  const int gb = b0[w.inst] + w.lb;
  block_chunks<V, X, Acc>(rp, ci, val, x, chunk_row, chunk_cls, bchunk[gb], bchunk[gb + 1],
                          [&](int) { return NoPre{}; }, [&](int i, Acc s, NoPre) { y[i] = Y(s); });
}

// The same product over a layout whose blocks are (first, end) chunk pairs (the A-side iteration
// layout; its long-row blocks have no chunks).
template <typename V, typename X, typename Acc, typename Y>
__global__ __launch_bounds__(kBlock) void k_spmv_pairs(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                       const V *__restrict__ val, const int32_t *__restrict__ chunk_row,
                                                       const int8_t *__restrict__ chunk_cls,
                                                       const int32_t *__restrict__ b0, const int32_t *__restrict__ binst,
                                                       const int32_t *__restrict__ bpair, const X *__restrict__ x,
                                                       Y *__restrict__ y) {
  const WBlock w = work_block(b0, binst);
  const int gb = b0[w.inst] + w.lb;
  block_chunks<V, X, Acc>(rp, ci, val, x, chunk_row, chunk_cls, bpair[2 * gb], bpair[2 * gb + 1],
                          [&](int) { return NoPre{}; }, [&](int i, Acc s, NoPre) { y[i] = Y(s); });
}

// Balanced contiguous share [*lo, *hi) of `count` items for block lb of nb.
__device__ __forceinline__ void share(int base, int count, int lb, int nb, int *lo, int *hi) {
  *lo = base + (int)(((int64_t)lb * count) / nb);
  *hi = base + (int)(((int64_t)(lb + 1) * count) / nb);
}

// ----------------------------------------------------------------------------------------------
// Column-panel sums of A x for the long rows (FP32). Rows of 64 or more nonzeros gather their x
// values at random from the whole vector; served from L2 those gathers are bound by the number of
// requests a compute unit can keep in flight, not by bytes. Here a work group takes one row block
// and one panel of kPanelW consecutive columns: it copies that panel of x into LDS with coalesced
// loads, then sums each row's entries in the panel with LDS gathers (G lanes per row, four FP64
// accumulators per lane as in the chunk engine, then a G-lane shuffle tree) and writes the row's
// panel sum. The row's epilogue adds its panel sums in panel order (k_dual, k_long_sum). Every
// summation order is fixed by the layout, so results are deterministic.
// ----------------------------------------------------------------------------------------------
template <typename T, typename X>
__device__ __forceinline__ void panel_sums(const Layout &L, const Panels<T> &Q, const X *__restrict__ x,
                                           double *__restrict__ part, T *xs) {
  const int wg = blockIdx.x;
  const int rb = Q.wg_rb[wg], p = Q.wg_p[wg], q = Q.rb_inst[rb];
  const int c0 = L.col0[q] + p * kPanelW;
  const int cn = min(kPanelW, L.col0[q + 1] - c0);
  for (int i = (int)threadIdx.x; i < cn; i += kPanelBlock) xs[i] = T(x[c0 + i]);
  __syncthreads();
  const int R = Q.rb_R[rb], G = Q.rb_G[rb];
  const int64_t eb = Q.wg_ebase[wg];
  const uint16_t *__restrict__ off = Q.off + Q.wg_obase[wg];
  const uint16_t *__restrict__ col = Q.col + eb;
  const T *__restrict__ val = Q.val + eb;
  const int ng = kPanelBlock / G, g = (int)threadIdx.x / G, l = (int)threadIdx.x % G;
  const int Rq = L.lr_R[q];
  double *__restrict__ out = part + L.lr_base[q] + (int64_t)p * Rq + Q.rb_lrow0[rb];
  for (int r = g; r < R; r += ng) {  // the G lanes of a group run the same rows
    const int a = off[r], b = off[r + 1];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int e = a + l;
    // plain (cached) loads: with few lanes per row the four strided loads of a lane share cache
    // lines, which the streaming hint would fetch from L2 one load at a time (measured 25 % slower)
    for (; e + 3 * G < b; e += 4 * G) {
      const int k0 = col[e], k1 = col[e + G], k2 = col[e + 2 * G], k3 = col[e + 3 * G];
      const T v0 = val[e], v1 = val[e + G], v2 = val[e + 2 * G], v3 = val[e + 3 * G];
      s0 = acc_fma(s0, double(v0), double(xs[k0]));
      s1 = acc_fma(s1, double(v1), double(xs[k1]));
      s2 = acc_fma(s2, double(v2), double(xs[k2]));
      s3 = acc_fma(s3, double(v3), double(xs[k3]));
    }
    for (; e < b; e += G) s0 = acc_fma(s0, double(val[e]), double(xs[col[e]]));
    double s = (s0 + s1) + (s2 + s3);
    for (int d = G >> 1; d > 0; d >>= 1) s += __shfl_xor(s, d, kWave);
    if (l == 0) out[r] = s;
  }
}

// The panel sums of A x' of one PDHG attempt (launched before k_dual).
template <typename T>
__global__ __launch_bounds__(kPanelBlock) void k_panel(Iter<T> P, Panels<T> Q) {
  __shared__ T xs[kPanelW];
  const State *st = P.st + Q.rb_inst[Q.wg_rb[blockIdx.x]];
  if (st->done | st->stop) return;
  panel_sums<T, T>(P.L, Q, P.x[st->cur ^ 1], P.part, xs);
}

// The panel sums of A x for a given x (products outside the iteration, diagnostics).
template <typename T>
__global__ __launch_bounds__(kPanelBlock) void k_panel_x(Layout L, Panels<T> Q, const T *__restrict__ x,
                                                         double *__restrict__ part) {
  __shared__ T xs[kPanelW];
  panel_sums<T, T>(L, Q, x, part, xs);
}

// y_i = sum of row i's panel sums, for the long rows (grid: the A-side blocks of the iteration
// layout; the chunk blocks return).
template <typename Y>
__global__ __launch_bounds__(kBlock) void k_long_sum(Layout L, const double *__restrict__ part, Y *__restrict__ y) {
  const WBlock w = work_block(L.ab0, L.ab_inst);
  const int gb = L.ab0[w.inst] + w.lb;
  if (L.a_bchunk[2 * gb] >= 0) return;
  const int Rq = L.lr_R[w.inst], Pq = L.lr_P[w.inst], r0 = L.row0[w.inst];
  const double *__restrict__ pq = part + L.lr_base[w.inst];
  const int j = -1 - L.a_bchunk[2 * gb];
  const int rhi = min((j + 1) * kBlock, Rq);
  for (int r = j * kBlock + (int)threadIdx.x; r < rhi; r += kBlock) {
    double s = 0.0;
    for (int pn = 0; pn < Pq; ++pn) s += pq[(int64_t)pn * Rq + r];
    y[r0 + r] = Y(s);
  }
}

// ----------------------------------------------------------------------------------------------
// One PDHG attempt is three launches: k_dual, k_step, k_primal (k_panel first when a handle sums
// long rows by column panels). Block partial sums are finished
// by the per-instance k_step in the next launch, so no block ever needs a device-wide fence.
//
// k_dual: A x' fused with the dual update.
//   ax'_i = (A x')_i ;  y'_i = proj_Y(y_i + sigma (b_i - 2 ax'_i + ax_i)), sigma = eta * omega
//   per-block partial sums of |dy|^2 and dy'(ax' - ax).
// Grid: the A-side work blocks of all instances; each owns a contiguous run of chunks.
// ----------------------------------------------------------------------------------------------
template <typename T>
struct DualSide {
  struct Pre {
    T y, ax, b;
    uint8_t s;
  };
  int cur;
  double sigma;
  const T *__restrict__ yc;
  const T *__restrict__ axc;
  T *__restrict__ yn;
  T *__restrict__ axn;
  const T *__restrict__ b;
  const uint8_t *__restrict__ sense;

  __device__ __forceinline__ DualSide(const Iter<T> &P, const State *st) {
    cur = st->cur;
    sigma = st->eta * st->omega;
    yc = P.y[cur], axc = P.ax[cur], yn = P.y[cur ^ 1], axn = P.ax[cur ^ 1], b = P.b, sense = P.sense;
  }
  __device__ __forceinline__ Pre fetch(int i) const { return Pre{yc[i], axc[i], b[i], sense[i]}; }
  // row i given its sum s = (A x')_i: the dual candidate, and the row's share of |dy|^2 and dy'(ax' - ax).
  // The update is computed in FP64 from the stored operands and rounded once to T.
  __device__ __forceinline__ void row(int i, double s, const Pre &q, double (&acc)[2]) const {
    const T axi = T(s);
    const double ax1 = double(axi), ax0 = double(q.ax), y0 = double(q.y);
    const T ynew = T(proj_dual(y0 + sigma * (double(q.b) - 2.0 * ax1 + ax0), q.s));
    yn[i] = ynew;
    axn[i] = axi;
    const double dy = double(ynew) - y0;
    acc[0] += dy * dy;
    acc[1] += dy * (ax1 - ax0);
  }
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dual(Iter<T> P) {
  const int4 d = P.L.ia_desc[blockIdx.x];  // instance, chunk range, partial-pair slot: one load
  const int inst = d.x, c_lo = d.y;
  const State *st = P.st + inst;
  if (st->done | st->stop | P.L.rb_n[inst]) return;
  const DualSide<T> D(P, st);
  const T *__restrict__ xn = P.x[D.cur ^ 1];
  double acc[2] = {0.0, 0.0};
  auto pre = [&](int i) { return D.fetch(i); };
  auto epi = [&](int i, double s, const typename DualSide<T>::Pre &q) { D.row(i, s, q, acc); };
  if (c_lo >= 0) {
    block_chunks<T, T, double>(P.a_rp, P.a_ci, P.a_val, xn, P.a_chunk_row, P.a_chunk_cls, c_lo, d.z, pre, epi);
  } else {
    // long rows (column-panel path): the row sum is its panel sums added in panel order
    const int Rq = P.L.lr_R[inst], Pq = P.L.lr_P[inst], r0 = P.L.row0[inst];
    const double *__restrict__ part = P.part + P.L.lr_base[inst];
    const int j = -1 - c_lo;
    const int rhi = min((j + 1) * kBlock, Rq);
    for (int r = j * kBlock + (int)threadIdx.x; r < rhi; r += kBlock) {
      const typename DualSide<T>::Pre q = pre(r0 + r);
      // the panel sums are read eight at a time (all loads issued before the first add; one block
      // per kBlock long rows keeps few waves per compute unit) and added in panel order
      constexpr int kU = 8;
      double s = 0.0;
      for (int p0 = 0; p0 < Pq; p0 += kU) {
        double v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
          v[u] = p0 + u < Pq ? __builtin_nontemporal_load(part + (int64_t)(p0 + u) * Rq + r) : 0.0;
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (p0 + u < Pq) s += v[u];
      }
      epi(r0 + r, s, q);
    }
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    P.p_dual[2 * d.w] = acc[0];
    P.p_dual[2 * d.w + 1] = acc[1];
  }
}

// ----------------------------------------------------------------------------------------------
// k_step (one block per instance): the adaptive step-size rule.
//   eta_bar = (omega |dx|^2 + |dy|^2 / omega) / (2 |dy'(A dx)|), accept iff eta <= eta_bar,
//   eta <- min((1 - (k+1)^-0.3) eta_bar, (1 + (k+1)^-0.6) eta).
// |dx|^2 comes from the kernel that produced the primal candidate (k_primal, or k_restart after a
// restart or at start-up).
// ----------------------------------------------------------------------------------------------
__device__ inline void step_size_rule(State *st, int32_t *ndone, double dx2, double dy2, double inter) {
  const double eta = st->eta, omega = st->omega;
  const double denom = 2.0 * fabs(inter);
  const double eta_bar = denom > 0.0 ? (omega * dx2 + dy2 / omega) / denom : INFINITY;
  const int64_t k = st->k + 1;
  st->k = k;
  const double kk = (double)(k + 1);
  const double eta_new = fmin((1.0 - pow(kk, -0.3)) * eta_bar, (1.0 + pow(kk, -0.6)) * eta);
  if (eta <= eta_bar) {
    st->cur ^= 1;
    st->wsum += eta;
    const double w = eta / st->wsum;
    if (!st->pair_avg) {
      st->avg_w = w, st->avg_mode = kAvgOne;
    } else if (st->pend_w > 0.0) {
      st->avg_w1 = st->pend_w, st->avg_w = w, st->pend_w = 0.0, st->avg_mode = kAvgPair;
    } else {
      st->pend_w = w, st->avg_mode = kAvgDefer;
    }
    st->commit = 1;
  } else {
    st->commit = 0;
  }
  st->eta = eta_new;
  if (!isfinite(eta_new) || !(eta_new > 0.0)) {
    st->status = 3;  // PDLP_STATUS_NUMERICAL
    mark_done(st, ndone);
  } else if (k >= st->iter_limit && (k % st->eval_every) != 0) {
    st->status = 2;  // PDLP_STATUS_ITER_LIMIT
    st->stop = 1;
  }
}

// The three step-size sums in one pass: |dy|^2 and dy'(A dx) over p_dual[2 q], p_dual[2 q + 1],
// q in [a_lo, a_hi), and |dx|^2 over p_dx[q], q in [t_lo, t_hi). Each sum keeps the order of a
// single strided reduction (four accumulators per thread over q, q + B, q + 2B, q + 3B, a wave
// tree, then the waves in order), so the three loads chains overlap without changing any result.
// The partials were written by blocks on every XCD, so each load goes to memory: a thread first
// issues sixteen strides' loads and only then adds them, in the same order (accumulator u takes
// strides u, u + 4, u + 8, u + 12), to pay one round trip per sixteen strides instead of per four.
// Results valid in thread 0.
constexpr int kStepBlock = 1024;
__device__ __forceinline__ void step_sums(const double *__restrict__ p_dual, int a_lo, int a_hi,
                                          const double *__restrict__ p_dx, int t_lo, int t_hi, double &dy2,
                                          double &inter, double &dx2) {
  constexpr int B = kStepBlock;
  double a[3][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
  int q = a_lo + (int)threadIdx.x;
  for (; q + 15 * B < a_hi; q += 16 * B) {
    double v0[16], v1[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      v0[t] = p_dual[2 * (size_t)(q + t * B)];
      v1[t] = p_dual[2 * (size_t)(q + t * B) + 1];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep every load above the first add
#pragma unroll
    for (int t = 0; t < 16; ++t) a[0][t & 3] += v0[t], a[1][t & 3] += v1[t];
  }
  for (; q + 3 * B < a_hi; q += 4 * B) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[0][u] += p_dual[2 * (size_t)(q + u * B)];
      a[1][u] += p_dual[2 * (size_t)(q + u * B) + 1];
    }
  }
  for (; q < a_hi; q += B) a[0][0] += p_dual[2 * (size_t)q], a[1][0] += p_dual[2 * (size_t)q + 1];
  q = t_lo + (int)threadIdx.x;
  for (; q + 15 * B < t_hi; q += 16 * B) {
    double v2[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) v2[t] = p_dx[q + t * B];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 16; ++t) a[2][t & 3] += v2[t];
  }
  for (; q + 3 * B < t_hi; q += 4 * B) {
#pragma unroll
    for (int u = 0; u < 4; ++u) a[2][u] += p_dx[q + u * B];
  }
  for (; q < t_hi; q += B) a[2][0] += p_dx[q];
  __shared__ double red[3][B / kWave];
  double v[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = wave_sum((a[i][0] + a[i][1]) + (a[i][2] + a[i][3]));
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) red[i][threadIdx.x / kWave] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      v[i] = red[i][0];
      for (int w = 1; w < B / kWave; ++w) v[i] += red[i][w];
    }
    dy2 = v[0], inter = v[1], dx2 = v[2];
  }
}

__global__ __launch_bounds__(kStepBlock) void k_step(Layout L, const double *__restrict__ p_dual,
                                                     const double *__restrict__ p_primal,
                                                     const double *__restrict__ p_restart, State *sts,
                                                     int32_t *ndone) {
  const int inst = blockIdx.x;
  State *st = sts + inst;
  if (st->done) return;
  if (st->stop) {  // the pending commit was applied by k_primal / k_restart: finish
    if (threadIdx.x == 0) mark_done(st, ndone);
    return;
  }
  const bool rs = st->restart_mode != kNoRestart;
  double dy2 = 0.0, inter = 0.0, dx2 = 0.0;
  step_sums(p_dual, L.db0[inst], L.db0[inst + 1], rs ? p_restart : p_primal, rs ? L.ev_blk0[inst] : L.pb0[inst],
            rs ? L.ev_blk0[inst + 1] : L.pb0[inst + 1], dy2, inter, dx2);
  if (threadIdx.x == 0) {
    st->restart_mode = kNoRestart;
    step_size_rule(st, ndone, dx2, dy2, inter);
  }
}

// ----------------------------------------------------------------------------------------------
// k_primal: if the attempt was accepted, A'y' (committing it) and the weighted averages (x_bar,
// A'y_bar over the block's columns; y_bar, A x_bar over its share of the rows); then the primal
// candidate of the next attempt x' = proj_[l,u](x - tau (c - A'y)), tau = eta / omega, and its
// |x' - x|^2 partial sum. Grid: the A'-side work blocks of all instances.
// With paired averages (avg_mode) a deferred attempt leaves x_bar / y_bar alone, and the next
// accepted one applies the older update (its iterate is still in the other buffer: rejected
// candidates never overwrite the committed iterate) and then its own, per element, before the
// candidate of the next attempt overwrites that buffer.
// ----------------------------------------------------------------------------------------------
template <typename T>
struct PrimalSide {
  struct Pre {
    T x, c, l, u;
    double xbar;
    T atybar;
  };
  // FP64 keeps A'y-bar and A x-bar current with the averages' weighted updates; FP32 recomputes
  // both before each evaluation (the only readers), so it skips them here.
  static constexpr bool kTrack = sizeof(T) == sizeof(double);
  int cur, commit, stop, amode;
  bool avg_now;  // x_bar / y_bar change in this launch
  double tau, wad, wd1;
  T wa;
  const T *__restrict__ xc;
  T *__restrict__ xnx;
  const T *__restrict__ c;
  const T *__restrict__ lo;
  const T *__restrict__ hi;
  double *__restrict__ xbar;
  T *__restrict__ atybar;

  __device__ __forceinline__ PrimalSide(const Iter<T> &P, const State *st) {
    cur = st->cur, commit = st->commit, stop = st->stop, amode = st->avg_mode;
    avg_now = commit && amode != kAvgDefer;
    tau = st->eta / st->omega;
    wa = T(st->avg_w);
    wad = st->avg_w, wd1 = st->avg_w1;
    xc = P.x[cur], xnx = P.x[cur ^ 1], c = P.c, lo = P.l, hi = P.u, xbar = P.xbar, atybar = P.atybar;
  }
  __device__ __forceinline__ Pre fetch(int j) const {
    return Pre{xc[j], c[j], lo[j], hi[j], avg_now ? xbar[j] : 0.0, kTrack ? atybar[j] : T(0)};
  }
  // column j's share of the launch: averages (committed attempts) and the next primal candidate
  __device__ __forceinline__ void column(int j, T atyj, const Pre &q, double &dx2) const {
    if (commit) {
      if (amode == kAvgOne) {
        xbar[j] = q.xbar + wad * (double(q.x) - q.xbar);
      } else if (amode == kAvgPair) {
        const double t = q.xbar + wd1 * (double(xnx[j]) - q.xbar);
        xbar[j] = t + wad * (double(q.x) - t);
      }
      if (kTrack) atybar[j] = q.atybar + wa * (atyj - q.atybar);
    }
    if (!stop) {
      const T xnew = T(clipv(double(q.x) - tau * (double(q.c) - double(atyj)), double(q.l), double(q.u)));
      xnx[j] = xnew;
      const double d = double(xnew) - double(q.x);
      dx2 += d * d;
    }
  }
  // the dual averages of a committed attempt over rows [rb, re), thread t taking rb + t, + stride ...
  __device__ __forceinline__ void rows(const Iter<T> &P, int rb, int re, int t, int stride) const {
    if (!(avg_now || kTrack)) return;
    const T *__restrict__ yc = P.y[cur];
    const T *__restrict__ axc = P.ax[cur];
    const T *__restrict__ yprev = P.y[cur ^ 1];  // the older accepted y of a paired update
    double *__restrict__ ybar = P.ybar;
    T *__restrict__ axbar = P.axbar;
    for (int i = rb + t; i < re; i += stride) {
      if (amode == kAvgOne) {
        ybar[i] += wad * (double(yc[i]) - ybar[i]);
      } else if (amode == kAvgPair) {
        const double u = ybar[i] + wd1 * (double(yprev[i]) - ybar[i]);
        ybar[i] = u + wad * (double(yc[i]) - u);
      }
      if (kTrack) axbar[i] += wa * (axc[i] - axbar[i]);
    }
  }
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_primal(Iter<T> P) {
  // instance, chunk range, partial slot and share of the rows: two loads issued together
  const int4 d = P.L.tb_desc[blockIdx.x];
  const int2 rr = P.L.tb_rows[blockIdx.x];
  const int inst = d.x, cb = d.y, ce = d.z;
  const State *st = P.st + inst;
  if (st->done || P.L.cb_n[inst] > 0) return;
  const PrimalSide<T> S(P, st);
  T *__restrict__ aty = P.aty;
  double acc[1] = {0.0};
  auto fetch = [&](int j) { return S.fetch(j); };
  if (S.commit) {
    block_chunks<T, T, double>(P.t_rp, P.t_ci, P.t_val, P.y[S.cur], P.t_chunk_row, P.t_chunk_cls, cb, ce, fetch,
                               [&](int j, double s, const typename PrimalSide<T>::Pre &q) {
                                 const T atyj = T(s);
                                 aty[j] = atyj;
                                 S.column(j, atyj, q, acc[0]);
                               });
    S.rows(P, rr.x, rr.y, (int)threadIdx.x, kBlock);
  } else if (!S.stop && ce > cb) {
    const int j0 = P.t_chunk_row[cb], j1 = P.t_chunk_row[ce];
    for (int j = j0 + (int)threadIdx.x; j < j1; j += kBlock) S.column(j, aty[j], S.fetch(j), acc[0]);
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) P.p_primal[d.w] = acc[0];
}

// ----------------------------------------------------------------------------------------------
// Column-block path of A'y (FP32 instances whose columns are short and spread over all rows, so
// that every entry gathers y from a random row). Served from L2 such gathers are bound by the
// requests a compute unit can keep in flight, not by bytes. Here a work group owns kCbCols
// consecutive columns and walks y in row panels of kCbRows entries held in LDS. Its waves take the
// 64-lane groups of runs of the current panel (layout in ColBlocks): a lane sums its run in row
// order in FP64 (the product of two FP32 values is exact in FP64, so each step rounds once) and
// adds the run's sum to the column's FP64 accumulator in LDS. A column has one run per panel and
// panels are separated by barriers, so each column receives its panel sums in panel order and the
// result depends on the layout alone. While a panel is summed, the next panel's y values and the
// wave's first groups of it are loaded into registers. Rows are stored longest first, so the first
// panels hold most entries; later panels would cost a panel step (one memory latency) for a few
// entries each, so the entries past the dense panels (the tail) form one run per column that
// gathers y directly and is added last. The layout is streamed with non-temporal loads, like the
// chunk engine's, so that it does not evict the A-side panel data from the last-level cache
// between attempts.
// ----------------------------------------------------------------------------------------------
// v0: [K + 1] offsets of the gathered vector per instance (rows for A'y, columns for A x).
template <typename T>
__device__ __forceinline__ void cb_sums(const int32_t *__restrict__ v0, const ColBlocks<T> &Q, int wg,
                                        const T *__restrict__ y, float *ys, double *acc, int32_t *gsl, int32_t *ebl) {
  static_assert(sizeof(T) == sizeof(float), "the column-block path holds FP32 y panels in LDS");
  constexpr int kW = kCbBlock / kWave;     // waves per work group
  constexpr int kYr = kCbRows / kCbBlock;  // y values per thread and panel
  constexpr int kGb = 4;                   // groups per wave and panel held in registers
  // a panel has at most kCbCols runs, so kGb groups per wave cover all of them
  static_assert(kGb * kW * kWave >= kCbCols, "every group of a panel must have a register slot");
  const int q = Q.wg_inst[wg];
  const int r0 = v0[q], mq = v0[q + 1] - r0;
  const int np = Q.ndense[q];
  const uint32_t *__restrict__ desc = Q.desc;
  const uint16_t *__restrict__ rows = Q.row;
  const T *__restrict__ val = Q.val;
  const int tid = (int)threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  for (int i = tid; i < kCbCols; i += kCbBlock) acc[i] = 0.0;
  // the work group's group ranges and entry bases, in LDS
  {
    const int32_t *__restrict__ g = Q.gstart + Q.wg_g0[wg];
    for (int i = tid; i <= np; i += kCbBlock) gsl[i] = g[i];
    __syncthreads();
    const int gf = gsl[0], gn = gsl[np] - gf;
    for (int i = tid; i < gn; i += kCbBlock) ebl[i] = Q.ebase[gf + i];
    __syncthreads();
  }
  const int gfirst = gsl[0];
  // registers of the next panel: y values, and descriptors and first two slots of the wave's
  // groups
  float yr[kYr];
  uint32_t dr[kGb], rr0[kGb], rr1[kGb];
  float vr0[kGb], vr1[kGb];
  auto load = [&](int p) {
    const int rp0 = r0 + p * kCbRows, rn = min(kCbRows, mq - p * kCbRows);
#pragma unroll
    for (int u = 0; u < kYr; ++u) {
      const int i = tid + u * kCbBlock;
      yr[u] = i < rn ? float(y[rp0 + i]) : 0.0f;
    }
    const int g0 = gsl[p] + wave, g1 = gsl[p + 1];
#pragma unroll
    for (int u = 0; u < kGb; ++u) {
      const int g = g0 + u * kW;
      if (g < g1) {
        const int64_t e = (int64_t)ebl[g - gfirst] * kWave + lane;
        dr[u] = __builtin_nontemporal_load(desc + (int64_t)g * kWave + lane);
        rr0[u] = __builtin_nontemporal_load(rows + e), vr0[u] = float(__builtin_nontemporal_load(val + e));
        rr1[u] = __builtin_nontemporal_load(rows + e + kWave);
        vr1[u] = float(__builtin_nontemporal_load(val + e + kWave));
      }
    }
  };
  // one group: lane l sums its run (first two slots given) and adds the sum to its column
  auto run = [&](int g, uint32_t d, uint32_t ra, float va, uint32_t rb, float vb) {
    const int len = (int)(d >> 16), lc = (int)(d & 0xFFFFu);
    const int glen = __builtin_amdgcn_readfirstlane(len);  // the group's first run is its longest
    double s = 0.0;
    if (len > 0) s = fma(double(va), double(ys[ra]), s);
    if (len > 1) s = fma(double(vb), double(ys[rb]), s);
    // the remaining slots eight at a time: the loads of a batch are issued together, then summed
    // in order (runs in the densest panel are tens of entries long)
    constexpr int kB = 8;
    const int64_t e = (int64_t)ebl[g - gfirst] * kWave + lane;
    for (int t0 = 2; t0 < glen; t0 += kB) {
      uint32_t rq[kB];
      float vq[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        if (t0 + u < glen) {
          rq[u] = __builtin_nontemporal_load(rows + e + (int64_t)(t0 + u) * kWave);
          vq[u] = float(__builtin_nontemporal_load(val + e + (int64_t)(t0 + u) * kWave));
        }
      }
#pragma unroll
      for (int u = 0; u < kB; ++u)
        if (t0 + u < len) s = fma(double(vq[u]), double(ys[rq[u]]), s);
    }
    if (len > 0) acc[lc] += s;
  };
  if (np > 0) load(0);
  for (int p = 0; p < np; ++p) {
    const int rn = min(kCbRows, mq - p * kCbRows);
    const int g0 = gsl[p] + wave, g1 = gsl[p + 1];
    __syncthreads();  // the previous panel has been summed (and the accumulators cleared)
#pragma unroll
    for (int u = 0; u < kYr; ++u) {
      const int i = tid + u * kCbBlock;
      if (i < rn) ys[i] = yr[u];
    }
    uint32_t dc[kGb], rc0[kGb], rc1[kGb];
    float vc0[kGb], vc1[kGb];
#pragma unroll
    for (int u = 0; u < kGb; ++u) dc[u] = dr[u], rc0[u] = rr0[u], vc0[u] = vr0[u], rc1[u] = rr1[u], vc1[u] = vr1[u];
    __syncthreads();
    if (p + 1 < np) load(p + 1);
#pragma unroll
    for (int u = 0; u < kGb; ++u)
      if (g0 + u * kW < g1) run(g0 + u * kW, dc[u], rc0[u], vc0[u], rc1[u], vc1[u]);
  }
  __syncthreads();  // the last panel's sums are in the accumulators
  // the tail: one run per column, y gathered from memory, eight slots (loads, then gathers) at a time
  {
    constexpr int kB = 8;
    const int t1 = Q.wg_t[wg + 1];
    for (int g = Q.wg_t[wg] + wave; g < t1; g += kW) {
      const uint32_t d = __builtin_nontemporal_load(Q.tdesc + (int64_t)g * kWave + lane);
      const int64_t e = (int64_t)Q.tebase[g] * kWave + lane;
      const int len = (int)(d >> 16), lc = (int)(d & 0xFFFFu);
      const int glen = __builtin_amdgcn_readfirstlane(len);  // the group's first run is its longest
      double s = 0.0;
      for (int t0 = 0; t0 < glen; t0 += kB) {
        int32_t rq[kB];
        float vq[kB], yq[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          if (t0 + u < glen) {
            rq[u] = __builtin_nontemporal_load(Q.trow + e + (int64_t)(t0 + u) * kWave);
            vq[u] = float(__builtin_nontemporal_load(Q.tval + e + (int64_t)(t0 + u) * kWave));
          }
        }
#pragma unroll
        for (int u = 0; u < kB; ++u)
          if (t0 + u < len) yq[u] = float(y[r0 + rq[u]]);
#pragma unroll
        for (int u = 0; u < kB; ++u)
          if (t0 + u < len) s = fma(double(vq[u]), double(yq[u]), s);
      }
      if (len > 0) acc[lc] += s;
    }
  }
  __syncthreads();
}

// Sum over the block (kCbBlock threads) in a fixed order; valid in thread 0.
__device__ __forceinline__ double cb_block_sum(double v, double *red) {
  constexpr int kW = kCbBlock / kWave;
  v = wave_sum(v);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < kW; ++w) t += red[w];
    v = t;
  }
  return v;
}

// k_primal for the instances on the column-block path (grid: their work groups).
template <typename T>
__global__ __launch_bounds__(kCbBlock) void k_primal_cb(Iter<T> P, ColBlocks<T> Q) {
  __shared__ float ys[kCbRows];
  __shared__ double acc[kCbCols];
  __shared__ int32_t gsl[kCbMaxPanels + 1];
  __shared__ int32_t ebl[kCbMaxGroups];
  __shared__ double red[kCbBlock / kWave];
  const int wg = blockIdx.x, q = Q.wg_inst[wg], blk = Q.wg_blk[wg];
  const State *st = P.st + q;
  if (st->done) return;
  const PrimalSide<T> S(P, st);
  const int c0 = P.L.col0[q] + blk * kCbCols, cn = min(kCbCols, P.L.col0[q + 1] - c0);
  const int tid = (int)threadIdx.x;
  double dx2 = 0.0;
  if (S.commit) {
    cb_sums<T>(P.L.row0, Q, wg, P.y[S.cur], ys, acc, gsl, ebl);
    for (int i = tid; i < cn; i += kCbBlock) {
      const int j = c0 + i;
      const typename PrimalSide<T>::Pre pre = S.fetch(j);
      const T atyj = T(acc[i]);
      P.aty[j] = atyj;
      S.column(j, atyj, pre, dx2);
    }
    int rb, re;
    share(P.L.row0[q], P.L.row0[q + 1] - P.L.row0[q], blk, P.L.cb_n[q], &rb, &re);
    S.rows(P, rb, re, tid, kCbBlock);
  } else if (!S.stop) {
    for (int i = tid; i < cn; i += kCbBlock) S.column(c0 + i, P.aty[c0 + i], S.fetch(c0 + i), dx2);
  }
  dx2 = cb_block_sum(dx2, red);
  if (tid == 0) P.p_primal[P.L.pb0[q] + blk] = dx2;
}

// A'y for a given y over the column-block instances (plain store; products outside the iteration).
template <typename T>
__global__ __launch_bounds__(kCbBlock) void k_cb_x(Layout L, ColBlocks<T> Q, const T *__restrict__ y,
                                                   T *__restrict__ out) {
  __shared__ float ys[kCbRows];
  __shared__ double acc[kCbCols];
  __shared__ int32_t gsl[kCbMaxPanels + 1];
  __shared__ int32_t ebl[kCbMaxGroups];
  const int wg = blockIdx.x, q = Q.wg_inst[wg], blk = Q.wg_blk[wg];
  const int c0 = L.col0[q] + blk * kCbCols, cn = min(kCbCols, L.col0[q + 1] - c0);
  cb_sums<T>(L.row0, Q, wg, y, ys, acc, gsl, ebl);
  for (int i = (int)threadIdx.x; i < cn; i += kCbBlock) out[c0 + i] = T(acc[i]);
}

// Row blocks of A (FP32; the mirror of column blocks): a work group owns kCbCols consecutive rows
// of an instance and walks x in panels of kCbRows columns held in LDS; each row's entries in a panel
// form a run (in column order) summed by one lane, the runs past the dense panels gathered (layout
// and summation as in cb_sums, with rows as the lines and columns as the positions). Then the dual
// update of each of the work group's rows and its (|dy|^2, dy'(A dx)) partial pair, as k_dual.
template <typename T>
__global__ __launch_bounds__(kCbBlock) void k_dual_rb(Iter<T> P, ColBlocks<T> R) {
  __shared__ float xs[kCbRows];
  __shared__ double acc[kCbCols];
  __shared__ int32_t gsl[kCbMaxPanels + 1];
  __shared__ int32_t ebl[kCbMaxGroups];
  __shared__ double red[2 * (kCbBlock / kWave)];
  const int wg = blockIdx.x, q = R.wg_inst[wg], blk = R.wg_blk[wg];
  const State *st = P.st + q;
  if (st->done | st->stop) return;
  const DualSide<T> D(P, st);
  cb_sums<T>(P.L.col0, R, wg, P.x[D.cur ^ 1], xs, acc, gsl, ebl);
  const int i0 = P.L.row0[q] + blk * kCbCols, rn = min(kCbCols, P.L.row0[q + 1] - i0);
  const int tid = (int)threadIdx.x;
  double a2[2] = {0.0, 0.0};
  for (int i = tid; i < rn; i += kCbBlock) D.row(i0 + i, acc[i], D.fetch(i0 + i), a2);
  constexpr int kW = kCbBlock / kWave;
#pragma unroll
  for (int v = 0; v < 2; ++v) a2[v] = wave_sum(a2[v]);
  if ((tid & (kWave - 1)) == 0) red[tid / kWave] = a2[0], red[kW + tid / kWave] = a2[1];
  __syncthreads();
  if (tid == 0) {
    double s0 = red[0], s1 = red[kW];
    for (int w = 1; w < kW; ++w) s0 += red[w], s1 += red[kW + w];
    const int slot = P.L.db0[q] + blk;
    P.p_dual[2 * slot] = s0;
    P.p_dual[2 * slot + 1] = s1;
  }
}

// A x for a given x over the row-block instances (plain store; products outside the iteration).
template <typename T>
__global__ __launch_bounds__(kCbBlock) void k_rb_x(Layout L, ColBlocks<T> R, const T *__restrict__ x,
                                                   T *__restrict__ out) {
  __shared__ float xs[kCbRows];
  __shared__ double acc[kCbCols];
  __shared__ int32_t gsl[kCbMaxPanels + 1];
  __shared__ int32_t ebl[kCbMaxGroups];
  const int wg = blockIdx.x, q = R.wg_inst[wg], blk = R.wg_blk[wg];
  const int i0 = L.row0[q] + blk * kCbCols, rn = min(kCbCols, L.row0[q + 1] - i0);
  cb_sums<T>(L.col0, R, wg, x, xs, acc, gsl, ebl);
  for (int i = (int)threadIdx.x; i < rn; i += kCbBlock) out[i0 + i] = T(acc[i]);
}

// ----------------------------------------------------------------------------------------------
// Evaluation every eval_every attempts, on the committed current iterate and the average:
// residuals in scaled and original space, objectives, distances to the restart anchor (FP64).
// k_eval writes block partials; k_eval_fin (one block per instance) applies termination, the
// restart test and the primal weight update. Grid of k_eval: the evaluation blocks.
// ----------------------------------------------------------------------------------------------
struct Cand {
  double rp2, rp2o, by, dya2, rd2, rd2o, bt, cx, dxa2;
};

__device__ __forceinline__ void cand_errors(const Cand &q, double omega, double nb, double nc,
                                            double &rel_p, double &rel_d, double &rel_gap,
                                            double &pobj, double &dobj, double &kkt_w) {
  pobj = q.cx;
  dobj = q.by + q.bt;
  const double gap = pobj - dobj;
  rel_p = sqrt(q.rp2o) / (1.0 + nb);
  rel_d = sqrt(q.rd2o) / (1.0 + nc);
  rel_gap = fabs(gap) / (1.0 + fabs(pobj) + fabs(dobj));
  kkt_w = sqrt(omega * omega * q.rp2 + q.rd2 / (omega * omega) + gap * gap);
}

__device__ inline void eval_logic(State *st, int32_t *ndone, const double *tot, int mode) {
  Cand qc{tot[0], tot[1], tot[2], tot[3], tot[4], tot[5], tot[6], tot[7], tot[8]};
  Cand qa{tot[9], tot[10], tot[11], tot[12], tot[13], tot[14], tot[15], tot[16], tot[17]};
  double omega = st->omega;
  double rc[5], ra[5], kwc, kwa;
  cand_errors(qc, omega, st->nb, st->nc, rc[0], rc[1], rc[2], rc[3], rc[4], kwc);
  cand_errors(qa, omega, st->nb, st->nc, ra[0], ra[1], ra[2], ra[3], ra[4], kwa);
  const double kc = fmax(rc[0], fmax(rc[1], rc[2]));
  const double ka = fmax(ra[0], fmax(ra[1], ra[2]));
  st->cand_rel[0] = kc;
  st->cand_rel[1] = ka;
  for (int q = 0; q < 3; ++q) st->ev_rel[q] = rc[q], st->ev_rel[3 + q] = ra[q];
  if (mode != kEvalChunk) {
    st->rel_p = rc[0], st->rel_d = rc[1], st->rel_gap = rc[2], st->pobj = rc[3], st->dobj = rc[4];
    if (mode == kEvalInit) {
      st->kkt_anchor = kwc;
      st->kkt_prev = INFINITY;
    }
    return;
  }
  if (!isfinite(kc) && !isfinite(ka)) {
    st->status = 3;
    mark_done(st, ndone);
    return;
  }
  const bool pass_c = kc <= st->tol, pass_a = ka <= st->tol;
  if (pass_c || pass_a) {
    const int which = (pass_a && (!pass_c || ka < kc)) ? 1 : 0;
    const double *r = which ? ra : rc;
    st->rel_p = r[0], st->rel_d = r[1], st->rel_gap = r[2], st->pobj = r[3], st->dobj = r[4];
    st->which = which;
    st->status = 1;
    mark_done(st, ndone);
    return;
  }
  const bool use_avg = kwa < kwc;
  const double kkt_c = use_avg ? kwa : kwc;
  const int64_t k = st->k;
  const int64_t t_since = k - st->last_restart;
  const bool restart = (kkt_c <= 0.2 * st->kkt_anchor) ||
                       (kkt_c <= 0.8 * st->kkt_anchor && kkt_c > st->kkt_prev) ||
                       ((double)t_since >= 0.36 * (double)k);
  if (!restart) {
    st->kkt_prev = kkt_c;
    st->restart_mode = kNoRestart;
  } else {
    const Cand &q = use_avg ? qa : qc;
    const double ddx = sqrt(q.dxa2), ddy = sqrt(q.dya2);
    if (ddx > 1e-10 && ddy > 1e-10) omega = exp(0.5 * log(ddy / ddx) + 0.5 * log(omega));
    st->omega = omega;
    double t0, t1, t2, t3, t4, kw;
    cand_errors(q, omega, st->nb, st->nc, t0, t1, t2, t3, t4, kw);
    st->kkt_anchor = kw;
    st->kkt_prev = INFINITY;
    st->wsum = 0.0;
    st->last_restart = k;
    st->restarts += 1;
    st->restart_mode = use_avg ? kToAverage : kToCurrent;
  }
  if (k >= st->iter_limit) {
    st->status = 2;
    st->rel_p = rc[0], st->rel_d = rc[1], st->rel_gap = rc[2], st->pobj = rc[3], st->dobj = rc[4];
    st->which = 0;
    if (st->restart_mode == kNoRestart) mark_done(st, ndone);
    else st->stop = 1;
  }
}

// Instance of an evaluation-type block and its local block index / count.
struct EvBlock {
  int inst, lb, nlb;
};
__device__ __forceinline__ EvBlock ev_block(const Layout &L) {
  EvBlock e;
  e.inst = L.ev_inst[blockIdx.x];
  const int b0 = L.ev_blk0[e.inst];
  e.lb = (int)blockIdx.x - b0;
  e.nlb = L.ev_blk0[e.inst + 1] - b0;
  return e;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_eval(Iter<T> P) {
  const EvBlock E = ev_block(P.L);
  const State *st = P.st + E.inst;
  if (st->done) return;
  const int cur = st->cur;
  double a[kEvalNV];
#pragma unroll
  for (int q = 0; q < kEvalNV; ++q) a[q] = 0.0;
  const int gs = E.nlb * kBlock, off = E.lb * kBlock + (int)threadIdx.x;
  const T *__restrict__ yc = P.y[cur];
  const T *__restrict__ axc = P.ax[cur];
  const int r1 = P.L.row0[E.inst + 1];
  for (int i = P.L.row0[E.inst] + off; i < r1; i += gs) {
    const double b = double(P.b[i]), dr = P.Dr[i], ya = double(P.ya[i]);
    const uint8_t s = P.sense[i];
    {
      const double y = double(yc[i]);
      const double t = row_violation(b - double(axc[i]), s);
      const double to = t / dr, d = y - ya;
      a[0] += t * t, a[1] += to * to, a[2] += b * y, a[3] += d * d;
    }
    {
      const double y = double(P.ybar[i]);
      const double t = row_violation(b - double(P.axbar[i]), s);
      const double to = t / dr, d = y - ya;
      a[9] += t * t, a[10] += to * to, a[11] += b * y, a[12] += d * d;
    }
  }
  const T *__restrict__ xc = P.x[cur];
  const int c1 = P.L.col0[E.inst + 1];
  for (int j = P.L.col0[E.inst] + off; j < c1; j += gs) {
    const double c = double(P.c[j]), lo = double(P.l[j]), hi = double(P.u[j]);
    const double dc = P.Dc[j], xa = double(P.xa[j]);
    {
      const double x = double(xc[j]), g = c - double(P.aty[j]);
      const double lam = proj_reduced(g, lo, hi), rd = g - lam, rdo = rd / dc, d = x - xa;
      a[4] += rd * rd, a[5] += rdo * rdo, a[6] += bound_term(lo, hi, lam), a[7] += c * x, a[8] += d * d;
    }
    {
      const double x = double(P.xbar[j]), g = c - double(P.atybar[j]);
      const double lam = proj_reduced(g, lo, hi), rd = g - lam, rdo = rd / dc, d = x - xa;
      a[13] += rd * rd, a[14] += rdo * rdo, a[15] += bound_term(lo, hi, lam), a[16] += c * x, a[17] += d * d;
    }
  }
  block_sum<kEvalNV>(a);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kEvalNV; ++q) P.p_eval[(size_t)blockIdx.x * kEvalNV + q] = a[q];
  }
}

__global__ __launch_bounds__(kBlock) void k_eval_fin(Layout L, const double *__restrict__ p_eval, State *sts,
                                                     int32_t *ndone, int mode) {
  State *st = sts + blockIdx.x;
  if (st->done) return;
  double tot[kEvalNV];
  final_sum<kEvalNV>(p_eval, L.ev_blk0[blockIdx.x], L.ev_blk0[blockIdx.x + 1], tot);
  if (threadIdx.x == 0) {
    st->pend_w = 0.0;  // k_avg_flush has applied a pending average update before this evaluation
    eval_logic(st, ndone, tot, mode);
  }
}

// Before an evaluation reads the averages: apply the update an accepted attempt left pending
// (paired averages). No accepted attempt followed it, so its iterate is the committed one.
// Grid: the evaluation blocks.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_avg_flush(Iter<T> P) {
  const EvBlock E = ev_block(P.L);
  const State *st = P.st + E.inst;
  if (st->done) return;
  const double w = st->pend_w;
  if (!(w > 0.0)) return;
  const int cur = st->cur;
  const T *__restrict__ xc = P.x[cur];
  const T *__restrict__ yc = P.y[cur];
  const int gs = E.nlb * kBlock, off = E.lb * kBlock + (int)threadIdx.x;
  for (int j = P.L.col0[E.inst] + off; j < P.L.col0[E.inst + 1]; j += gs)
    P.xbar[j] = P.xbar[j] + w * (double(xc[j]) - P.xbar[j]);
  for (int i = P.L.row0[E.inst] + off; i < P.L.row0[E.inst + 1]; i += gs)
    P.ybar[i] += w * (double(yc[i]) - P.ybar[i]);
}

// ----------------------------------------------------------------------------------------------
// Restart (also used once at start-up with kToCurrent): move the chosen candidate into the current
// iterate, make it the anchor and the new average, then recompute the primal candidate with the
// possibly new primal weight; its |x' - x|^2 partials go to p_restart (k_step reads them while
// restart_mode is set). Grid: the evaluation blocks.
// ----------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restart(Iter<T> P) {
  const EvBlock E = ev_block(P.L);
  const State *st = P.st + E.inst;
  if (st->done) return;
  const int mode = st->restart_mode;
  if (mode == kNoRestart) return;
  const int cur = st->cur, stop = st->stop;
  const double tau = st->eta / st->omega;
  T *__restrict__ xc = P.x[cur];
  T *__restrict__ xnx = P.x[cur ^ 1];
  T *__restrict__ yc = P.y[cur];
  T *__restrict__ axc = P.ax[cur];
  double acc[1] = {0.0};
  const int gs = E.nlb * kBlock, off = E.lb * kBlock + (int)threadIdx.x;
  const int c1 = P.L.col0[E.inst + 1];
  for (int j = P.L.col0[E.inst] + off; j < c1; j += gs) {
    T xj, atyj;
    if (mode == kToAverage) {
      xj = T(P.xbar[j]), atyj = P.atybar[j];
      xc[j] = xj, P.aty[j] = atyj;
    } else {
      xj = xc[j], atyj = P.aty[j];
      P.xbar[j] = xj, P.atybar[j] = atyj;
    }
    P.xa[j] = xj;
    if (!stop) {
      const T xnew = T(clipv(double(xj) - tau * (double(P.c[j]) - double(atyj)), double(P.l[j]), double(P.u[j])));
      xnx[j] = xnew;
      const double d = double(xnew) - double(xj);
      acc[0] += d * d;
    }
  }
  const int r1 = P.L.row0[E.inst + 1];
  for (int i = P.L.row0[E.inst] + off; i < r1; i += gs) {
    T yi;
    if (mode == kToAverage) {
      yi = T(P.ybar[i]);
      yc[i] = yi, axc[i] = P.axbar[i];
    } else {
      yi = yc[i];
      P.ybar[i] = yi, P.axbar[i] = axc[i];
    }
    P.ya[i] = yi;
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) P.p_restart[blockIdx.x] = acc[0];
}

// ----------------------------------------------------------------------------------------------
// Start point: x = proj_[l~,u~](x0 / Dc or 0), y = proj_Y(y0 / Dr or 0), rounded once to T.
// ----------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_point(int m, int n, const double *__restrict__ x0,
                                                       const double *__restrict__ y0, const double *__restrict__ Dr,
                                                       const double *__restrict__ Dc, const double *__restrict__ l64,
                                                       const double *__restrict__ u64,
                                                       const uint8_t *__restrict__ sense, T *__restrict__ x,
                                                       T *__restrict__ y) {
  const int gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
  for (int j = gt; j < n; j += gs) x[j] = T(clipv(x0 ? x0[j] / Dc[j] : 0.0, l64[j], u64[j]));
  for (int i = gt; i < m; i += gs) y[i] = T(proj_dual(y0 ? y0[i] / Dr[i] : 0.0, sense[i]));
}

// ----------------------------------------------------------------------------------------------
// Finalize: select each instance's returned point (current or average), unscale it, and recompute
// its residuals in FP64 from the FP64 scaled matrix (ax64 = A~ x~, aty64 = A~' y~ computed by
// k_spmv in FP64 in between). Grid: the evaluation blocks; k_final_fin: one block per instance.
// ----------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_unscale(Iter<T> P, double *__restrict__ xd, double *__restrict__ yd,
                                                    double *__restrict__ x_out, double *__restrict__ y_out) {
  const EvBlock E = ev_block(P.L);
  const State *st = P.st + E.inst;
  const int cur = st->cur, which = st->which;
  const T *__restrict__ x = P.x[cur];
  const T *__restrict__ y = P.y[cur];
  const int gs = E.nlb * kBlock, off = E.lb * kBlock + (int)threadIdx.x;
  for (int j = P.L.col0[E.inst] + off; j < P.L.col0[E.inst + 1]; j += gs) {
    const double v = which ? P.xbar[j] : double(x[j]);
    xd[j] = v;
    x_out[j] = P.Dc[j] * v;
  }
  for (int i = P.L.row0[E.inst] + off; i < P.L.row0[E.inst + 1]; i += gs) {
    const double v = which ? P.ybar[i] : double(y[i]);
    yd[i] = v;
    y_out[i] = P.Dr[i] * v;
  }
}

struct Final64 {
  const double *xd, *yd, *ax64, *aty64, *c64, *b64, *l64, *u64;
  double *rc_out;
  double *p_final;
};
template <typename T>
__global__ __launch_bounds__(kBlock) void k_final_residuals(Iter<T> P, Final64 F) {
  const EvBlock E = ev_block(P.L);
  double a[5] = {0, 0, 0, 0, 0};  // rp2o, rd2o, by, bt, cx
  const int gs = E.nlb * kBlock, off = E.lb * kBlock + (int)threadIdx.x;
  for (int i = P.L.row0[E.inst] + off; i < P.L.row0[E.inst + 1]; i += gs) {
    const double t = row_violation(F.b64[i] - F.ax64[i], P.sense[i]) / P.Dr[i];
    a[0] += t * t;
    a[2] += F.b64[i] * F.yd[i];
  }
  for (int j = P.L.col0[E.inst] + off; j < P.L.col0[E.inst + 1]; j += gs) {
    const double g = F.c64[j] - F.aty64[j];
    const double lam = proj_reduced(g, F.l64[j], F.u64[j]);
    const double rdo = (g - lam) / P.Dc[j];
    a[1] += rdo * rdo;
    a[3] += bound_term(F.l64[j], F.u64[j], lam);
    a[4] += F.c64[j] * F.xd[j];
    F.rc_out[j] = g / P.Dc[j];
  }
  block_sum<5>(a);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 5; ++q) F.p_final[(size_t)blockIdx.x * 5 + q] = a[q];
  }
}

__global__ __launch_bounds__(kBlock) void k_final_fin(Layout L, const double *__restrict__ p_final, State *sts) {
  State *st = sts + blockIdx.x;
  double tot[5];
  final_sum<5>(p_final, L.ev_blk0[blockIdx.x], L.ev_blk0[blockIdx.x + 1], tot);
  if (threadIdx.x == 0) {
    const double pobj = tot[4], dobj = tot[2] + tot[3];
    st->rel_p = sqrt(tot[0]) / (1.0 + st->nb);
    st->rel_d = sqrt(tot[1]) / (1.0 + st->nc);
    st->rel_gap = fabs(pobj - dobj) / (1.0 + fabs(pobj) + fabs(dobj));
    st->pobj = pobj;
    st->dobj = dobj;
  }
}

// ----------------------------------------------------------------------------------------------
// Per-instance FP64 reductions used during set-up, one block per instance segment [s0[k], s0[k+1]):
// kind 0 = sum of squares, kind 1 = max |v|.
// ----------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_seg_reduce(int kind, const int32_t *__restrict__ s0,
                                                       const double *__restrict__ v, double *__restrict__ out) {
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int i = s0[k] + (int)threadIdx.x; i < s0[k + 1]; i += kBlock) {
    const double t = v[i];
    acc = kind == 0 ? acc + t * t : fmax(acc, fabs(t));
  }
  __shared__ double red[kWaves];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const double o = __shfl_xor(acc, off, kWave);
    acc = kind == 0 ? acc + o : fmax(acc, o);
  }
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < kWaves; ++w) r = kind == 0 ? r + red[w] : fmax(r, red[w]);
    out[k] = r;
  }
}

// ----------------------------------------------------------------------------------------------
// Set-up: transpose by counting sort (histogram, exclusive scan, scatter, per-column sort of the
// scattered source positions so the result is deterministic, gather).
// ----------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_expand_rows(int m, const int32_t *__restrict__ rp, int32_t *__restrict__ row_of) {
  // one wave per row
  const int wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int lane = threadIdx.x % kWave;
  const int nwaves = gridDim.x * kWaves;
  for (int i = wave; i < m; i += nwaves)
    for (int e = rp[i] + lane; e < rp[i + 1]; e += kWave) row_of[e] = i;
}

__global__ __launch_bounds__(kBlock) void k_histogram(int nnz, const int32_t *__restrict__ ci, int32_t *__restrict__ cnt) {
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < nnz; e += gridDim.x * kBlock) atomicAdd(&cnt[ci[e]], 1);
}

// Exclusive scan of in[0..n) into out[0..n], out[n] = total. Blocks of kScanItems items.
constexpr int kScanPer = 8;
constexpr int kScanItems = kBlock * kScanPer;

__device__ __forceinline__ int block_exclusive_scan(int v, int *total) {
  __shared__ int wsum[kWaves];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  int inc = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int t = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += t;
  }
  __syncthreads();
  if (lane == kWave - 1) wsum[wid] = inc;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < wid) base += wsum[w];
    tot += wsum[w];
  }
  *total = tot;
  return base + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_partial(int n, const int32_t *__restrict__ in, int32_t *__restrict__ bsum) {
  const int base = blockIdx.x * kScanItems + threadIdx.x * kScanPer;
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q)
    if (base + q < n) s += in[base + q];
  int tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_bsums(int nb, int32_t *__restrict__ bsum) {
  int carry = 0;
  for (int off = 0; off < nb; off += kBlock) {
    const int i = off + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    int tot;
    const int ex = block_exclusive_scan(v, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_final(int n, const int32_t *__restrict__ in, const int32_t *__restrict__ bsum,
                                                       int32_t *__restrict__ out) {
  if (n == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
    return;
  }
  const int base = blockIdx.x * kScanItems + threadIdx.x * kScanPer;
  int v[kScanPer];
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    v[q] = base + q < n ? in[base + q] : 0;
    s += v[q];
  }
  int tot;
  int run = block_exclusive_scan(s, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanPer; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
  if (base <= n - 1 && n - 1 < base + kScanPer) out[n] = run;  // thread holding the last item
}

__global__ __launch_bounds__(kBlock) void k_scatter(int nnz, const int32_t *__restrict__ ci, const int32_t *__restrict__ t_rp,
                                                    int32_t *__restrict__ fill, int32_t *__restrict__ perm) {
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < nnz; e += gridDim.x * kBlock) {
    const int j = ci[e];
    const int p = t_rp[j] + atomicAdd(&fill[j], 1);
    perm[p] = e;
  }
}

// Sort every segment of length <= 32 in place (one thread per segment, insertion sort).
__global__ __launch_bounds__(kBlock) void k_segsort_small(int nseg, const int32_t *__restrict__ sp, int32_t *__restrict__ d) {
  for (int s = blockIdx.x * kBlock + threadIdx.x; s < nseg; s += gridDim.x * kBlock) {
    const int a = sp[s], b = sp[s + 1];
    if (b - a > 32 || b - a < 2) continue;
    for (int i = a + 1; i < b; ++i) {
      const int key = d[i];
      int j = i - 1;
      while (j >= a && d[j] > key) {
        d[j + 1] = d[j];
        --j;
      }
      d[j + 1] = key;
    }
  }
}

// Bitonic sort of the listed long segments, one block per segment. Segments whose padded length
// fits kSortLds are sorted in LDS, longer ones in their slice of `scratch` (offset scr_off[q]).
constexpr int kSortLds = 4096;
__device__ void bitonic(int32_t *buf, int N) {
  for (int k = 2; k <= N; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += kBlock) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          const int a = buf[i], b = buf[ixj];
          if ((a > b) == up) {
            buf[i] = b;
            buf[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_segsort_large(const int32_t *__restrict__ seg_list, const int32_t *__restrict__ sp,
                                                          int32_t *__restrict__ d, int32_t *__restrict__ scratch,
                                                          const int64_t *__restrict__ scr_off) {
  __shared__ int32_t lbuf[kSortLds];
  const int s = seg_list[blockIdx.x];
  const int a = sp[s], len = sp[s + 1] - a;
  int N = 1;
  while (N < len) N <<= 1;
  int32_t *buf = N <= kSortLds ? lbuf : scratch + scr_off[blockIdx.x];
  for (int i = threadIdx.x; i < N; i += kBlock) buf[i] = i < len ? d[a + i] : INT32_MAX;
  __syncthreads();
  bitonic(buf, N);
  for (int i = threadIdx.x; i < len; i += kBlock) d[a + i] = buf[i];
}

// t_ci[p] = row of source entry perm[p]; t_val[p] = val[perm[p]]
template <typename V>
__global__ __launch_bounds__(kBlock) void k_gather_t(int nnz, const int32_t *__restrict__ perm, const int32_t *__restrict__ row_of,
                                                     const V *__restrict__ val, int32_t *__restrict__ t_ci, V *__restrict__ t_val) {
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < nnz; p += gridDim.x * kBlock) {
    const int e = perm[p];
    if (t_ci) t_ci[p] = row_of[e];
    t_val[p] = val[e];
  }
}

// out[p] = val[src[p]], or 0 where src[p] < 0
template <typename V>
__global__ __launch_bounds__(kBlock) void k_gather_or_zero(int64_t count, const int32_t *__restrict__ src,
                                                           const V *__restrict__ val, V *__restrict__ out) {
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < count; p += (int64_t)gridDim.x * kBlock) {
    const int32_t e = src[p];
    out[p] = e >= 0 ? val[e] : V(0);
  }
}

// ----------------------------------------------------------------------------------------------
// Set-up: equilibration. One wave per row reduces |a| (max or sum) over a row of A (direct) or a
// row of A' (values gathered through perm).
// ----------------------------------------------------------------------------------------------
template <bool kSum>
__global__ __launch_bounds__(kBlock) void k_row_norm(int rows, const int32_t *__restrict__ rp, const int32_t *__restrict__ perm,
                                                     const double *__restrict__ val, double *__restrict__ out) {
  const int wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int lane = threadIdx.x % kWave;
  const int nwaves = gridDim.x * kWaves;
  for (int r = wave; r < rows; r += nwaves) {
    double acc = 0.0;
    for (int e = rp[r] + lane; e < rp[r + 1]; e += kWave) {
      const double v = fabs(val[perm ? perm[e] : e]);
      acc = kSum ? acc + v : fmax(acc, v);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
      const double o = __shfl_xor(acc, off, kWave);
      acc = kSum ? acc + o : fmax(acc, o);
    }
    if (lane == 0) out[r] = acc > 0.0 ? sqrt(acc) : 1.0;
  }
}

// a_ij <- a_ij / (rho_i * kap_j); Dr /= rho; Dc /= kap
__global__ __launch_bounds__(kBlock) void k_apply_scale(int nnz, const int32_t *__restrict__ row_of, const int32_t *__restrict__ ci,
                                                        double *__restrict__ val, const double *__restrict__ rho,
                                                        const double *__restrict__ kap) {
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < nnz; e += gridDim.x * kBlock)
    val[e] = val[e] / (rho[row_of[e]] * kap[ci[e]]);
}

__global__ __launch_bounds__(kBlock) void k_div_inplace(int n, double *__restrict__ d, const double *__restrict__ s) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) d[i] = d[i] / s[i];
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, double *__restrict__ d, double v) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) d[i] = v;
}

// c~ = Dc c, l~ = l / Dc, u~ = u / Dc (infinite bounds stay infinite); b~ = Dr b. FP64 copies kept,
// T copies rounded once.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_vectors(int m, int n, const double *__restrict__ c, const double *__restrict__ l,
                                                          const double *__restrict__ u, const double *__restrict__ b,
                                                          const double *__restrict__ Dr, const double *__restrict__ Dc,
                                                          double *__restrict__ c64, double *__restrict__ l64,
                                                          double *__restrict__ u64, double *__restrict__ b64, T *__restrict__ cT,
                                                          T *__restrict__ lT, T *__restrict__ uT, T *__restrict__ bT) {
  const int gt = blockIdx.x * kBlock + threadIdx.x, gs = gridDim.x * kBlock;
  for (int j = gt; j < n; j += gs) {
    const double cs = Dc[j] * c[j];
    const double ls = isfinite(l[j]) ? l[j] / Dc[j] : l[j];
    const double us = isfinite(u[j]) ? u[j] / Dc[j] : u[j];
    c64[j] = cs, l64[j] = ls, u64[j] = us;
    cT[j] = T(cs), lT[j] = T(ls), uT[j] = T(us);
  }
  for (int i = gt; i < m; i += gs) {
    const double bs = Dr[i] * b[i];
    b64[i] = bs;
    bT[i] = T(bs);
  }
}

// New bounds of one instance (columns c0 .. c0 + nq - 1 in internal numbering), scaled exactly as
// k_scale_vectors scales them at create time.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale_bounds(int nq, int c0, const double *__restrict__ l,
                                                         const double *__restrict__ u, const double *__restrict__ Dc,
                                                         double *__restrict__ l64, double *__restrict__ u64,
                                                         T *__restrict__ lT, T *__restrict__ uT) {
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < nq; k += gridDim.x * kBlock) {
    const int j = c0 + k;
    const double ls = isfinite(l[k]) ? l[k] / Dc[j] : l[k];
    const double us = isfinite(u[k]) ? u[k] / Dc[j] : u[k];
    l64[j] = ls, u64[j] = us;
    lT[j] = T(ls), uT[j] = T(us);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_convert(int64_t n, const double *__restrict__ s, T *__restrict__ d) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) d[i] = T(s[i]);
}

// dst[i] = src[idx[i]] (boundary mapping between external and internal numbering)
__global__ __launch_bounds__(kBlock) void k_gather64(int n, const double *__restrict__ src, const int32_t *__restrict__ idx,
                                                     double *__restrict__ dst) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) dst[i] = src[idx[i]];
}

// Original-space product helper: xs = x / D (scaled input, rounded to T) and y = ys / D.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_div_to(int n, const double *__restrict__ x, const double *__restrict__ D,
                                                   T *__restrict__ out) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) out[i] = T(x[i] / D[i]);
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_div_from(int n, const T *__restrict__ y, const double *__restrict__ D,
                                                     double *__restrict__ out) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) out[i] = double(y[i]) / D[i];
}

}  // namespace pdlp
