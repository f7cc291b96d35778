// Device kernels of the LP-based variable strategies and LP-based fixing (section 2 of the paper,
// "LP-based variable strategies", "LP-based fixing", "Tiebreaking and hybrid strategies").
//
// An order is a stable sort of the binary and integer variables (compacted in index order) by a list
// of keys, applied least significant first, so equal keys keep the lower index first. Every key is
// mapped to unsigned words whose ascending order is the wanted order:
//   Frac     fractionality f = min(x - floor x, ceil x - x) >= 0: the bits of f (ascending)
//   RedCost  |r|: the complement of the bits of |r| (descending)
//   Dual     the rank of the first constraint, in descending |y|, holding the variable (ascending),
//            then RedCost
//   Type     the variable type code, binary 1 before integer 2
// The sort is an LSD radix sort over 8-bit digits. Each pass: per-tile digit histograms, one
// exclusive scan over (digit, tile), then a stable scatter in which a tile is walked in 256-item
// rounds and each item's rank among equal digits of its wave comes from eight ballots.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdlp {
namespace fix {

constexpr int kSortBlock = 256;  // threads of every sort / scan block
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kSortRounds = 16;  // 256-item rounds per tile
constexpr int kSortTile = kSortBlock * kSortRounds;
constexpr int kDigits = 256;
constexpr int kScanPer = 16;  // items per thread in the local scan
constexpr int kScanTile = kSortBlock * kScanPer;
static_assert(kSortBlock == kDigits, "one thread per digit in the histogram and offset steps");

enum KeyKind : int { kKeyFrac = 0, kKeyRedCost = 1, kKeyRowDual = 2, kKeyGroup = 3, kKeyType = 4 };

__device__ __forceinline__ uint64_t key_bits(int kind, int32_t j, const double *__restrict__ x,
                                             const double *__restrict__ rc, const double *__restrict__ y,
                                             const uint8_t *__restrict__ vt, const uint32_t *__restrict__ group) {
  switch (kind) {
    case kKeyFrac: {
      const double v = x[j];
      const double f = fmin(v - floor(v), ceil(v) - v);
      return (uint64_t)__double_as_longlong(f);
    }
    case kKeyRedCost:
      return ~(uint64_t)__double_as_longlong(fabs(rc[j]));
    case kKeyRowDual:
      return ~(uint64_t)__double_as_longlong(fabs(y[j]));
    case kKeyGroup:
      return group[j];
    default:
      return vt[j];
  }
}

// keys[p] = word `word` (0 low, 1 high) of the key of item J[p]
__global__ __launch_bounds__(kSortBlock) void k_fix_key(int k, const int32_t *__restrict__ J, int kind, int word,
                                                        const double *__restrict__ x, const double *__restrict__ rc,
                                                        const double *__restrict__ y, const uint8_t *__restrict__ vt,
                                                        const uint32_t *__restrict__ group, uint32_t *__restrict__ keys) {
  for (int64_t p = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; p < k; p += (int64_t)gridDim.x * kSortBlock) {
    const uint64_t b = key_bits(kind, J[p], x, rc, y, vt, group);
    keys[p] = word ? (uint32_t)(b >> 32) : (uint32_t)b;
  }
}

// Per-tile histogram of one digit; counts are digit-major: counts[d * nb + tile].
__global__ __launch_bounds__(kSortBlock) void k_radix_hist(int n, const uint32_t *__restrict__ keys, int shift, int nb,
                                                           int32_t *__restrict__ counts) {
  __shared__ int32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t p = t0 + (int64_t)r * kSortBlock + threadIdx.x;
    if (p < n) atomicAdd(&h[(keys[p] >> shift) & 255u], 1);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one digit. offs = exclusive scan of the digit-major counts (the first output slot
// of each (digit, tile)). Within a round, items of a wave with equal digits are ranked by lane with
// eight ballots; waves follow in order, rounds follow in order, so the tile's order is kept. All of
// the tile's keys are loaded up front (one memory latency, not one per round), and the per-wave digit
// counts alternate between two buffers so that a round needs two barriers.
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(int n, int shift, int nb,
                                                              const uint32_t *__restrict__ kin,
                                                              const int32_t *__restrict__ vin,
                                                              const int32_t *__restrict__ offs,
                                                              uint32_t *__restrict__ kout, int32_t *__restrict__ vout) {
  __shared__ int32_t run[kDigits];
  __shared__ int32_t wcnt[2][kSortWaves][kDigits];
  const int t = (int)threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
  uint32_t kr[kSortRounds];
  int32_t vr[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t p = t0 + (int64_t)r * kSortBlock + t;
    kr[r] = p < n ? kin[p] : 0u;
    vr[r] = p < n ? vin[p] : 0;
  }
  run[t] = offs[(int64_t)t * nb + blockIdx.x];
#pragma unroll
  for (int v = 0; v < kSortWaves; ++v) wcnt[0][v][t] = 0, wcnt[1][v][t] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    int32_t(*cnt)[kDigits] = wcnt[r & 1];
    const bool valid = t0 + (int64_t)r * kSortBlock + t < n;
    const int dig = (int)((kr[r] >> shift) & 255u);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int bit = (dig >> b) & 1;
      const uint64_t ones = __ballot(bit);
      peers &= bit ? ones : ~ones;
    }
    const int rank = __popcll(peers & ((1ull << lane) - 1ull));
    if (valid && rank == 0) cnt[w][dig] = __popcll(peers);
    __syncthreads();  // this round's counts are complete; run[] holds the previous rounds
    if (valid) {
      int before = 0;
      for (int v = 0; v < w; ++v) before += cnt[v][dig];
      const int64_t dst = (int64_t)run[dig] + before + rank;
      if (dst < n) {
        kout[dst] = kr[r];
        vout[dst] = vr[r];
      }
    }
    __syncthreads();  // every read of run[] and of this round's counts is done
    int add = 0;
#pragma unroll
    for (int v = 0; v < kSortWaves; ++v) add += cnt[v][t], cnt[v][t] = 0;
    run[t] += add;  // read by others only after the next round's first barrier
  }
}

// Exclusive scan of 256 per-thread values of a block; `total` receives the block's sum.
__device__ __forceinline__ int block_exclusive_scan(int v, int *lds, int &total) {
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  int s = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(s, o, 64);
    if (lane >= o) s += u;
  }
  if (lane == 63) lds[w] = s;
  __syncthreads();
  int base = 0;
  total = 0;
#pragma unroll
  for (int i = 0; i < kSortWaves; ++i) {
    const int u = lds[i];
    if (i < w) base += u;
    total += u;
  }
  __syncthreads();
  return base + s - v;
}

// Three-step exclusive scan of N int32 values: per-tile scan with tile sums, scan of the tile sums
// (one block), add the tile offsets.
__global__ __launch_bounds__(kSortBlock) void k_scan_local(int64_t N, const int32_t *__restrict__ in,
                                                           int32_t *__restrict__ out, int32_t *__restrict__ tsum) {
  __shared__ int lds[kSortWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int v[kScanPer];
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = base + i < N ? in[base + i] : 0;
    s += v[i];
  }
  int total;
  int run = block_exclusive_scan(s, lds, total);
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < N) out[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kSortBlock) void k_scan_top(int ntiles, int32_t *__restrict__ tsum) {
  __shared__ int lds[kSortWaves];
  const int per = (ntiles + kSortBlock - 1) / kSortBlock;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  int s = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < ntiles) s += tsum[b0 + i];
  int total;
  int run = block_exclusive_scan(s, lds, total);
  for (int i = 0; i < per; ++i)
    if (b0 + i < ntiles) {
      const int u = tsum[b0 + i];
      tsum[b0 + i] = run;
      run += u;
    }
}

__global__ __launch_bounds__(kSortBlock) void k_scan_add(int64_t N, int32_t *__restrict__ out,
                                                         const int32_t *__restrict__ tsum) {
  for (int64_t p = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; p < N; p += (int64_t)gridDim.x * kSortBlock)
    out[p] += tsum[p / kScanTile];
}

// Compaction of the binary and integer variables, in index order.
__global__ __launch_bounds__(kSortBlock) void k_int_flags(int n, const uint8_t *__restrict__ vt, int32_t *__restrict__ f) {
  for (int64_t j = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kSortBlock)
    f[j] = vt[j] != 0;
}
__global__ __launch_bounds__(kSortBlock) void k_int_compact(int n, const uint8_t *__restrict__ vt,
                                                            const int32_t *__restrict__ pos, int32_t *__restrict__ J) {
  for (int64_t j = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kSortBlock)
    if (vt[j]) J[pos[j]] = (int32_t)j;
}

__global__ __launch_bounds__(kSortBlock) void k_iota(int n, int32_t *__restrict__ v) {
  for (int64_t j = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kSortBlock)
    v[j] = (int32_t)j;
}

// rank[R[p]] = p: position of each row in the descending-|y| order.
__global__ __launch_bounds__(kSortBlock) void k_rank(int m, const int32_t *__restrict__ R, int32_t *__restrict__ rank) {
  for (int64_t p = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; p < m; p += (int64_t)gridDim.x * kSortBlock)
    rank[R[p]] = (int32_t)p;
}

// Dual grouping over the stored transpose (internal numbering): a binary or integer variable's group
// is the smallest rank of a constraint holding it, m when its column is empty. Long columns (the
// first internal columns: columns are sorted by descending length class) take one wave each, the
// rest one thread each; the minimum does not depend on the order it is taken in.
constexpr int kLongColumn = 32;
__global__ __launch_bounds__(kSortBlock) void k_dual_group_long(int ncols, int m, const int32_t *__restrict__ t_rp,
                                                                const int32_t *__restrict__ t_ci,
                                                                const int32_t *__restrict__ perm_r,
                                                                const int32_t *__restrict__ perm_c,
                                                                const uint8_t *__restrict__ vt,
                                                                const int32_t *__restrict__ rank,
                                                                uint32_t *__restrict__ group) {
  const int lane = (int)threadIdx.x & 63;
  const int64_t wave0 = ((int64_t)blockIdx.x * kSortBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kSortBlock) >> 6;
  for (int64_t jj = wave0; jj < ncols; jj += nwaves) {
    const int32_t j = perm_c[jj];
    if (!vt[j]) continue;  // uniform over the wave
    int32_t g = m;
    for (int32_t e = t_rp[jj] + lane; e < t_rp[jj + 1]; e += 64) g = min(g, rank[perm_r[t_ci[e]]]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) g = min(g, __shfl_xor(g, o, 64));
    if (lane == 0) group[j] = (uint32_t)g;
  }
}

__global__ __launch_bounds__(kSortBlock) void k_dual_group(int first, int n, int m, const int32_t *__restrict__ t_rp,
                                                           const int32_t *__restrict__ t_ci,
                                                           const int32_t *__restrict__ perm_r,
                                                           const int32_t *__restrict__ perm_c,
                                                           const uint8_t *__restrict__ vt,
                                                           const int32_t *__restrict__ rank,
                                                           uint32_t *__restrict__ group) {
  for (int64_t jj = (int64_t)first + (int64_t)blockIdx.x * kSortBlock + threadIdx.x; jj < n;
       jj += (int64_t)gridDim.x * kSortBlock) {
    const int32_t j = perm_c[jj];
    if (!vt[j]) continue;
    int32_t g = m;
    for (int32_t e = t_rp[jj]; e < t_rp[jj + 1]; ++e) g = min(g, rank[perm_r[t_ci[e]]]);
    group[j] = (uint32_t)g;
  }
}

// LP-based fixing: floor x if the sample exceeds x - floor x, else ceil x, clamped to the integral
// part of the bounds; continuous variables keep x.
__global__ __launch_bounds__(kSortBlock) void k_lp_fixing(int n, const double *__restrict__ x,
                                                          const double *__restrict__ l, const double *__restrict__ u,
                                                          const uint8_t *__restrict__ vt,
                                                          const double *__restrict__ s, double *__restrict__ out) {
  for (int64_t j = (int64_t)blockIdx.x * kSortBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kSortBlock) {
    const double v = x[j];
    if (!vt[j]) {
      out[j] = v;
      continue;
    }
    const double lo = floor(v), hi = ceil(v);
    double a = s[j] > v - lo ? lo : hi;
    a = fmin(fmax(a, ceil(l[j])), floor(u[j]));
    out[j] = a;
  }
}

}  // namespace fix
}  // namespace pdlp
