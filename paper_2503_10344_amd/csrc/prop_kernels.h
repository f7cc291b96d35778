// Device kernels of linear-constraint bound propagation (the propagator fix-and-propagate applies
// after each fixing; section 2 of the paper names it without defining it, so this is the standard
// activity-based bound strengthening, run in Jacobi rounds).
//
// One round: every row reads the bounds of the round's start (l, u), forms its minimum and maximum
// activity in row order (finite part plus a count of infinite terms) and proposes, for each of its
// variables, the bound the other terms leave room for; a bound takes the tightest accepted proposal
// (atomic min / max on the bit pattern, so the result does not depend on the order rows finish in).
// Integer variables round proposals inward within 1e-6 and take any strict gain; continuous ones
// take a gain above 1e-3 max(1, |bound|). A second kernel then records whether a bound moved and
// whether some lower bound passed its upper bound.
//
// A column's two bounds are kept together (Bounds, 16 bytes): a row reads both bounds of each of its
// columns, so one 16-byte gather per nonzero replaces two 8-byte ones.
//
// Products and sums round separately: every function below switches floating-point contraction
// off (HIP contracts a * b + c into a fused multiply-add by default, and that rounds once instead of
// twice), so a row's activity is the same double as a plain sequential sum.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdlp {
namespace prop {

constexpr int kPropBlock = 256;
constexpr double kFeasTol = 1e-6;
constexpr double kContTol = 1e-3;

__device__ __forceinline__ void atomic_min_double(double *addr, double v) {
  unsigned long long *a = reinterpret_cast<unsigned long long *>(addr);
  unsigned long long old = __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (v < __longlong_as_double((long long)old)) {
    const unsigned long long seen = atomicCAS(a, old, (unsigned long long)__double_as_longlong(v));
    if (seen == old) break;
    old = seen;
  }
}
__device__ __forceinline__ void atomic_max_double(double *addr, double v) {
  unsigned long long *a = reinterpret_cast<unsigned long long *>(addr);
  unsigned long long old = __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (v > __longlong_as_double((long long)old)) {
    const unsigned long long seen = atomicCAS(a, old, (unsigned long long)__double_as_longlong(v));
    if (seen == old) break;
    old = seen;
  }
}

// New upper bound from a proposal p, or `cur` when it is not taken.
__device__ __forceinline__ double tighten_upper(double cur, double p, bool integral) {
#pragma clang fp contract(off)
  if (integral) {
    const double q = floor((p + kFeasTol));
    return q < cur ? q : cur;
  }
  if (isinf(cur)) return isinf(p) ? cur : p;
  return p < (cur - (kContTol * fmax(1.0, fabs(cur)))) ? p : cur;
}
__device__ __forceinline__ double tighten_lower(double cur, double p, bool integral) {
#pragma clang fp contract(off)
  if (integral) {
    const double q = ceil((p - kFeasTol));
    return q > cur ? q : cur;
  }
  if (isinf(cur)) return isinf(p) ? cur : p;
  return p > (cur + (kContTol * fmax(1.0, fabs(cur)))) ? p : cur;
}

constexpr int kLongRow = 128;  // rows at least this long are handled by a whole wave

struct alignas(16) Bounds {
  double lo, hi;
};

struct Activity {
  double minf, maxf;   // finite parts of the minimum / maximum activity, summed in row order
  int mininf, maxinf;  // infinite terms
};

// Activities of row [k0, k1) by one thread: the plain sequential sum.
__device__ __forceinline__ Activity activity_seq(int32_t k0, int32_t k1, const int32_t *__restrict__ ci,
                                                 const double *__restrict__ val,
                                                 const Bounds *__restrict__ lu) {
#pragma clang fp contract(off)
  Activity A{0.0, 0.0, 0, 0};
  for (int32_t k = k0; k < k1; ++k) {
    const double a = val[k];
    if (a == 0.0) continue;
    const int32_t j = ci[k];
    const Bounds bj = lu[j];
    const double lo = bj.lo, hi = bj.hi;
    const double tmin = a > 0.0 ? lo : hi, tmax = a > 0.0 ? hi : lo;
    if (isinf(tmin)) ++A.mininf;
    else A.minf = (A.minf + (a * tmin));
    if (isinf(tmax)) ++A.maxinf;
    else A.maxf = (A.maxf + (a * tmax));
  }
  return A;
}

// Lane t's value of v, for every lane (t uniform across the wave): a scalar read of that lane's
// register, without the LDS permute a general shuffle takes.
__device__ __forceinline__ int lane_value(int v, int t) { return __builtin_amdgcn_readlane(v, t); }
__device__ __forceinline__ double lane_value(double v, int t) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned int lo = (unsigned int)__builtin_amdgcn_readlane((int)(unsigned int)b, t);
  const unsigned int hi = (unsigned int)__builtin_amdgcn_readlane((int)(unsigned int)(b >> 32), t);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The same sum by a wave: each 64-element segment is loaded and multiplied by the lanes in parallel,
// then every lane adds the segment's terms in row order (broadcast one lane at a time by a scalar
// read of that lane), so all lanes end with the sequential sum's exact value without waiting on one
// gather per element.
__device__ __forceinline__ Activity activity_wave(int32_t k0, int32_t k1, int lane, const int32_t *__restrict__ ci,
                                                  const double *__restrict__ val,
                                                  const Bounds *__restrict__ lu) {
#pragma clang fp contract(off)
  Activity A{0.0, 0.0, 0, 0};
  for (int32_t seg = k0; seg < k1; seg += 64) {
    const int32_t k = seg + lane;
    double pmin = 0.0, pmax = 0.0;
    int code = 0;  // bit 0: a term exists (nonzero coefficient), bit 1: infinite min term, bit 2: infinite max term
    if (k < k1) {
      const double a = val[k];
      if (a != 0.0) {
        const int32_t j = ci[k];
        const Bounds bj = lu[j];
        const double lo = bj.lo, hi = bj.hi;
        const double tmin = a > 0.0 ? lo : hi, tmax = a > 0.0 ? hi : lo;
        code = 1 | (isinf(tmin) ? 2 : 0) | (isinf(tmax) ? 4 : 0);
        if (!isinf(tmin)) pmin = a * tmin;
        if (!isinf(tmax)) pmax = a * tmax;
      }
    }
    const int cnt = min(64, k1 - seg);
    for (int t = 0; t < cnt; ++t) {
      const int c = lane_value(code, t);
      if (c & 1) {
        if (c & 2) ++A.mininf;
        else A.minf = (A.minf + lane_value(pmin, t));
        if (c & 4) ++A.maxinf;
        else A.maxf = (A.maxf + lane_value(pmax, t));
      }
    }
  }
  return A;
}

// Proposals of one row from its activities, split over the lanes (first = lane, stride = lanes);
// flags[1] = 1 (from the first lane) when the row cannot be satisfied within the bounds: a finite
// activity past b by more than 1e-6 max(1, |b|).
__device__ __forceinline__ void prop_row(int64_t i, const Activity &A, int first, int stride,
                                         const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                         const double *__restrict__ val, const double *__restrict__ b,
                                         const uint8_t *__restrict__ sense, const uint8_t *__restrict__ vt,
                                         const Bounds *__restrict__ lu, Bounds *lun, int32_t *flags) {
#pragma clang fp contract(off)
  const int32_t k0 = rp[i], k1 = rp[i + 1];
  const double minf = A.minf, maxf = A.maxf;
  const int mininf = A.mininf, maxinf = A.maxinf;
  const double bi = b[i];
  const double tolb = (kFeasTol * fmax(1.0, fabs(bi)));
  const uint8_t s = sense[i];
  const bool le = s == 'L' || s == 'E', ge = s == 'G' || s == 'E';
  if (first == 0 && ((le && mininf == 0 && minf > (bi + tolb)) || (ge && maxinf == 0 && maxf < (bi - tolb))))
    atomicOr(&flags[1], 1);
  for (int32_t k = k0 + first; k < k1; k += stride) {
    const double a = val[k];
    if (a == 0.0) continue;
    const int32_t j = ci[k];
    const Bounds bj = lu[j];
    const double lo = bj.lo, hi = bj.hi;
    const bool integral = vt[j] != 0;
    if (le) {
      const double t = a > 0.0 ? lo : hi;
      bool ok = true;
      double res = 0.0;
      if (mininf == 0) res = (minf - (a * t));
      else if (mininf == 1 && isinf(t)) res = minf;
      else ok = false;
      if (ok) {
        const double p = (bi - res) / a;
        if (a > 0.0) {
          const double q = tighten_upper(hi, p, integral);
          if (q < hi) atomic_min_double(&lun[j].hi, q);
        } else {
          const double q = tighten_lower(lo, p, integral);
          if (q > lo) atomic_max_double(&lun[j].lo, q);
        }
      }
    }
    if (ge) {
      const double t = a > 0.0 ? hi : lo;
      bool ok = true;
      double res = 0.0;
      if (maxinf == 0) res = (maxf - (a * t));
      else if (maxinf == 1 && isinf(t)) res = maxf;
      else ok = false;
      if (ok) {
        const double p = (bi - res) / a;
        if (a > 0.0) {
          const double q = tighten_lower(lo, p, integral);
          if (q > lo) atomic_max_double(&lun[j].lo, q);
        } else {
          const double q = tighten_upper(hi, p, integral);
          if (q < hi) atomic_min_double(&lun[j].hi, q);
        }
      }
    }
  }
}

// Rows shorter than kLongRow: one thread each.
__global__ __launch_bounds__(kPropBlock) void k_prop_round(int m, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const double *__restrict__ val,
                                                           const double *__restrict__ b,
                                                           const uint8_t *__restrict__ sense,
                                                           const uint8_t *__restrict__ vt,
                                                           const Bounds *__restrict__ lu, Bounds *lun,
                                                           int32_t *flags) {
  for (int64_t i = (int64_t)blockIdx.x * kPropBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kPropBlock) {
    const int32_t k0 = rp[i], k1 = rp[i + 1];
    if (k1 - k0 >= kLongRow) continue;
    const Activity A = activity_seq(k0, k1, ci, val, lu);
    prop_row(i, A, 0, 1, rp, ci, val, b, sense, vt, lu, lun, flags);
  }
}

// Rows of at least kLongRow entries (listed in `rows`): one wave each.
__global__ __launch_bounds__(kPropBlock) void k_prop_round_long(int nlong, const int32_t *__restrict__ rows,
                                                                const int32_t *__restrict__ rp,
                                                                const int32_t *__restrict__ ci,
                                                                const double *__restrict__ val,
                                                                const double *__restrict__ b,
                                                                const uint8_t *__restrict__ sense,
                                                                const uint8_t *__restrict__ vt,
                                                                const Bounds *__restrict__ lu, Bounds *lun,
                                                                int32_t *flags) {
  const int lane = (int)threadIdx.x & 63;
  const int64_t wave0 = ((int64_t)blockIdx.x * kPropBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kPropBlock) >> 6;
  for (int64_t w = wave0; w < nlong; w += nwaves) {
    const int64_t i = rows[w];
    const Activity A = activity_wave(rp[i], rp[i + 1], lane, ci, val, lu);
    prop_row(i, A, lane, 64, rp, ci, val, b, sense, vt, lu, lun, flags);
  }
}

// After a round: flags[0] = 1 if a bound moved, flags[2] = 1 if some l > u + 1e-6; then the round's
// result becomes the current bounds (lu = lun), so both copies agree for the next round.
__global__ __launch_bounds__(kPropBlock) void k_prop_finish(int n, Bounds *__restrict__ lu,
                                                            const Bounds *__restrict__ lun, int32_t *flags) {
#pragma clang fp contract(off)
  bool moved = false, crossed = false;
  for (int64_t j = (int64_t)blockIdx.x * kPropBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kPropBlock) {
    const Bounds nx = lun[j], cu = lu[j];
    moved |= nx.lo != cu.lo || nx.hi != cu.hi;
    crossed |= nx.lo > (nx.hi + kFeasTol);
    lu[j] = nx;
  }
  // one atomic per block at most (and none once the flag is set): a round that moves millions of
  // bounds would otherwise queue one atomic per wave on the same address
  const int any_moved = __syncthreads_or(moved ? 1 : 0), any_crossed = __syncthreads_or(crossed ? 1 : 0);
  if (threadIdx.x == 0) {
    if (any_moved && __hip_atomic_load(&flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      atomicOr(&flags[0], 1);
    if (any_crossed) atomicOr(&flags[2], 1);
  }
}

// Both bound copies from the caller's l, u at the start of a call, and back at its end.
__global__ __launch_bounds__(kPropBlock) void k_prop_pack(int n, const double *__restrict__ l,
                                                          const double *__restrict__ u, Bounds *__restrict__ lu,
                                                          Bounds *__restrict__ lun) {
  for (int64_t j = (int64_t)blockIdx.x * kPropBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kPropBlock) {
    const Bounds v{l[j], u[j]};
    lu[j] = v;
    lun[j] = v;
  }
}
__global__ __launch_bounds__(kPropBlock) void k_prop_unpack(int n, const Bounds *__restrict__ lu,
                                                            double *__restrict__ l, double *__restrict__ u) {
  for (int64_t j = (int64_t)blockIdx.x * kPropBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kPropBlock) {
    const Bounds v = lu[j];
    l[j] = v.lo;
    u[j] = v.hi;
  }
}

}  // namespace prop
}  // namespace pdlp
