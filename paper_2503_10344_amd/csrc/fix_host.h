// Host side of the LP-based variable strategies and LP-based fixing: device workspace, the radix
// sort driver and the extern "C" entry points declared in include/pdlp_fix.h. Included at the end of
// pdlp.hip (it uses the solver handle, Arena, HIPCHK and guarded from there).
#pragma once

#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/pdlp_fix.h"
#include "fix_kernels.h"

namespace pdlp {
namespace fix {

static int fix_grid(int64_t n) {
  const int64_t g = (n + kSortBlock - 1) / kSortBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

// Device buffers kept in the handle between calls (fix-and-propagate asks for orders repeatedly):
// slot i grows when a call needs more, and the arena frees everything with the handle.
struct Cache {
  std::vector<std::pair<void *, int64_t>> slot;
};
struct Work {
  Arena &mem;
  Cache &c;
  int next = 0;
  Work(Arena &a, Cache &cache) : mem(a), c(cache) {}
  template <typename U>
  U *get(int64_t count) {
    const int64_t bytes = std::max<int64_t>(count, 1) * (int64_t)sizeof(U);
    if ((int)c.slot.size() <= next) c.slot.push_back({nullptr, 0});
    auto &e = c.slot[next++];
    if (e.second < bytes) {
      if (e.first) mem.release(e.first);
      e.first = nullptr, e.second = 0;
      e.first = mem.alloc<uint8_t>(bytes);
      e.second = bytes;
    }
    return static_cast<U *>(e.first);
  }
};
// Workspace carved from one caller-independent buffer (the allocation-free entry point): pieces
// aligned to 256 bytes, in call order; asking for more than the buffer holds raises before any
// kernel has been launched (every piece is taken at the start of a call).
struct ScratchWork {
  uint8_t *base;
  int64_t cap, used = 0;
  template <typename U>
  U *get(int64_t count) {
    const int64_t bytes = (std::max<int64_t>(count, 1) * (int64_t)sizeof(U) + 255) & ~(int64_t)255;
    if (used + bytes > cap)
      raise(PDLP_ERR_ARG, "problem too large for pdlp_variable_strategy_noalloc: its workspace exceeds the " +
                              std::to_string(cap >> 20) + " MiB static buffer (about 20.25 max(n, m) bytes, plus 4 n + 12 m with DUAL)");
    U *p = reinterpret_cast<U *>(base + used);
    used += bytes;
    return p;
  }
};

template <typename T>
Cache &cache_of(Solver<T> &s) {
  if (!s.fix_cache) s.fix_cache = std::make_shared<Cache>();
  return *static_cast<Cache *>(s.fix_cache.get());
}

// True for device (or managed) memory, false for ordinary host memory.
static bool on_device(const void *p) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// A device pointer to `count` values of `src`: src itself when it is device memory, else a copy.
// (The allocation-free path accepts device inputs only, so it never copies.)
template <typename U, typename W>
const U *device_input(W &w, const U *src, int64_t count, hipStream_t st) {
  if constexpr (std::is_same<W, ScratchWork>::value) return src;
  U *buf = w.template get<U>(count);  // taken in both cases so the slot numbering does not depend on it
  if (!src || count == 0) return buf;
  if (on_device(src)) return src;
  HIPCHK(hipMemcpyAsync(buf, src, sizeof(U) * (size_t)count, hipMemcpyHostToDevice, st));
  return buf;
}

// Stable LSD radix sort of (keys, vals) of n items by the low `digits` bytes of the keys. Buffers
// ping-pong between (k0, v0) and (k1, v1); on return (k0, v0) hold the result.
struct RadixSort {
  hipStream_t stream;
  int32_t *counts = nullptr, *offs = nullptr, *tsum = nullptr;
  void scan(int64_t N, const int32_t *in, int32_t *out) {
    const int64_t tiles = (N + kScanTile - 1) / kScanTile;
    if (tiles > (int64_t)kSortBlock * 1024) raise(PDLP_ERR_ARG, "scan too long");
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)tiles), dim3(kSortBlock), 0, stream, N, in, out, tsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kSortBlock), 0, stream, (int)tiles, tsum);
    hipLaunchKernelGGL(k_scan_add, dim3(fix_grid(N)), dim3(kSortBlock), 0, stream, N, out, (const int32_t *)tsum);
  }
  void sort(int n, int digits, uint32_t *&k0, int32_t *&v0, uint32_t *&k1, int32_t *&v1) {
    if (n <= 1) return;
    const int nb = (n + kSortTile - 1) / kSortTile;
    for (int d = 0; d < digits; ++d) {
      const int shift = 8 * d;
      hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortBlock), 0, stream, n, (const uint32_t *)k0, shift, nb,
                         counts);
      scan((int64_t)kDigits * nb, counts, offs);
      hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kSortBlock), 0, stream, n, shift, nb, (const uint32_t *)k0,
                         (const int32_t *)v0, (const int32_t *)offs, k1, v1);
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
    HIPCHK(hipGetLastError());
  }
};

// Key list of a strategy, most significant first.
static void strategy_keys(int s, std::vector<int> &keys) {
  switch (s) {
    case PDLP_ORDER_FRAC: keys.push_back(kKeyFrac); break;
    case PDLP_ORDER_REDCOST: keys.push_back(kKeyRedCost); break;
    case PDLP_ORDER_DUAL: keys.push_back(kKeyGroup), keys.push_back(kKeyRedCost); break;
    case PDLP_ORDER_TYPE: keys.push_back(kKeyType); break;
    default: break;
  }
}

static bool finite_host(const double *v, int64_t len) {
  for (int64_t i = 0; i < len; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// The order of one strategy. W supplies the device workspace: the handle's cache (grown on demand)
// or, for the allocation-free entry point, pieces of the static scratch buffer.
template <typename T, typename W>
void variable_strategy_in(Solver<T> &s, W &w, int strategy, int tiebreak, const uint8_t *var_type, const double *x,
                          const double *y, const double *rc, int32_t *order, int32_t *count) {
  const bool valid_s = strategy >= PDLP_ORDER_FRAC && strategy <= PDLP_ORDER_TYPE;
  const bool valid_t = tiebreak >= PDLP_ORDER_NONE && tiebreak <= PDLP_ORDER_TYPE;
  if (!valid_s || !valid_t) raise(PDLP_ERR_ARG, "unknown variable strategy or tiebreak");
  if (s.K != 1) raise(PDLP_ERR_ARG, "variable strategies take a single-problem handle");
  std::vector<int> keys;
  strategy_keys(strategy, keys);
  strategy_keys(tiebreak, keys);
  bool need_x = false, need_rc = false, need_y = false;
  for (int k : keys) need_x |= k == kKeyFrac, need_rc |= k == kKeyRedCost, need_y |= k == kKeyGroup;
  if (!var_type || !order || !count || (need_x && !x) || (need_rc && !rc) || (need_y && !y))
    raise(PDLP_ERR_ARG, "NULL argument that the strategy needs");
  const int n = s.n, m = s.m;
  // host inputs are checked here; device inputs must be finite
  if ((need_x && !on_device(x) && !finite_host(x, n)) || (need_rc && !on_device(rc) && !finite_host(rc, n)) ||
      (need_y && !on_device(y) && !finite_host(y, m)))
    raise(PDLP_ERR_ARG, "x, y and red_cost must be finite");
  hipStream_t st = s.stream;
  const int64_t big = std::max<int64_t>(std::max(n, m), 1);
  const uint8_t *d_vt = device_input(w, var_type, n, st);
  const double *d_x = device_input(w, need_x ? x : nullptr, need_x ? n : 0, st);
  const double *d_rc = device_input(w, need_rc ? rc : nullptr, need_rc ? n : 0, st);
  const double *d_y = device_input(w, need_y ? y : nullptr, need_y ? m : 0, st);
  uint32_t *k0 = w.template get<uint32_t>(big), *k1 = w.template get<uint32_t>(big);
  int32_t *v0 = w.template get<int32_t>(big), *v1 = w.template get<int32_t>(big);
  const int64_t max_tiles = (big + kSortTile - 1) / kSortTile;
  const int64_t scan_len = std::max<int64_t>((int64_t)kDigits * max_tiles, big);
  RadixSort rs{st};
  rs.counts = w.template get<int32_t>((int64_t)kDigits * max_tiles);
  rs.offs = w.template get<int32_t>(scan_len);
  rs.tsum = w.template get<int32_t>((scan_len + kScanTile - 1) / kScanTile + 1);
  uint32_t *d_group = w.template get<uint32_t>(need_y ? n : 0);
  int32_t *R0 = w.template get<int32_t>(need_y ? m : 0), *R1 = w.template get<int32_t>(need_y ? m : 0);
  int32_t *rank = w.template get<int32_t>(need_y ? m : 0);
  int32_t *tail = w.template get<int32_t>(2);

  // binary and integer variables, in index order
  int32_t k = 0;
  if (n) {
    hipLaunchKernelGGL(k_int_flags, dim3(fix_grid(n)), dim3(kSortBlock), 0, st, n, d_vt, v1);
    rs.scan(n, v1, rs.offs);
    hipLaunchKernelGGL(k_int_compact, dim3(fix_grid(n)), dim3(kSortBlock), 0, st, n, d_vt, (const int32_t *)rs.offs,
                       v0);
    int32_t h[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(tail, rs.offs + (n - 1), sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(tail + 1, v1 + (n - 1), sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(h, tail, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    k = h[0] + h[1];
  }

  // Dual: rank of each constraint in descending |y| (ties: lower index), then each variable's group
  if (need_y && k > 1) {
    if (m > 0) {
      hipLaunchKernelGGL(k_iota, dim3(fix_grid(m)), dim3(kSortBlock), 0, st, m, R0);
      for (int word = 0; word < 2; ++word) {
        hipLaunchKernelGGL(k_fix_key, dim3(fix_grid(m)), dim3(kSortBlock), 0, st, m, (const int32_t *)R0,
                           (int)kKeyRowDual, word, (const double *)nullptr, (const double *)nullptr, d_y,
                           (const uint8_t *)nullptr, (const uint32_t *)nullptr, k0);
        rs.sort(m, 4, k0, R0, k1, R1);
      }
      hipLaunchKernelGGL(k_rank, dim3(fix_grid(m)), dim3(kSortBlock), 0, st, m, (const int32_t *)R0, rank);
    }
    // internal columns are sorted by descending length class: the long ones form a prefix
    int nlong = 0;
    while (nlong < n && s.h_trp[nlong + 1] - s.h_trp[nlong] >= kLongColumn) ++nlong;
    if (nlong > 0)
      hipLaunchKernelGGL(k_dual_group_long, dim3(fix_grid((int64_t)nlong * 64)), dim3(kSortBlock), 0, st, nlong, m,
                         (const int32_t *)s.t_rp, (const int32_t *)s.t_ci, (const int32_t *)s.d_perm_r,
                         (const int32_t *)s.d_perm_c, d_vt, (const int32_t *)rank, d_group);
    if (nlong < n)
      hipLaunchKernelGGL(k_dual_group, dim3(fix_grid(n - nlong)), dim3(kSortBlock), 0, st, nlong, n, m,
                         (const int32_t *)s.t_rp, (const int32_t *)s.t_ci, (const int32_t *)s.d_perm_r,
                         (const int32_t *)s.d_perm_c, d_vt, (const int32_t *)rank, d_group);
  }

  // stable sorts, least significant key first
  const int group_digits = m < 256 ? 1 : m < 65536 ? 2 : m < (1 << 24) ? 3 : 4;
  for (int q = (int)keys.size() - 1; q >= 0 && k > 1; --q) {
    const int kind = keys[q];
    const bool wide = kind == kKeyFrac || kind == kKeyRedCost;
    const int digits = wide ? 4 : kind == kKeyGroup ? group_digits : 1;
    for (int word = 0; word < (wide ? 2 : 1); ++word) {
      hipLaunchKernelGGL(k_fix_key, dim3(fix_grid(k)), dim3(kSortBlock), 0, st, k, (const int32_t *)v0, kind, word,
                         d_x, d_rc, (const double *)nullptr, d_vt, (const uint32_t *)d_group, k0);
      rs.sort(k, digits, k0, v0, k1, v1);
    }
  }
  HIPCHK(hipGetLastError());
  if (k > 0) HIPCHK(hipMemcpyAsync(order, v0, sizeof(int32_t) * (size_t)k, hipMemcpyDefault, st));
  HIPCHK(hipStreamSynchronize(st));
  *count = k;
}

template <typename T>
void variable_strategy(Solver<T> &s, int strategy, int tiebreak, const uint8_t *var_type, const double *x,
                       const double *y, const double *rc, int32_t *order, int32_t *count) {
  Work w(s.mem, cache_of(s));
  variable_strategy_in(s, w, strategy, tiebreak, var_type, x, y, rc, order, count);
}

// ---------------------------------------------------------------------------------------------
// Allocation-free variant. Its workspace is one static device array per GPU, `scratch`; host code
// reaches it only through the address hipGetSymbolAddress returns for the current device (the
// array's name in host code is a host-side stand-in, not a device address). Every call on a GPU
// reuses that GPU's array, so two calls that overlap on one GPU race. No piece of the workspace is
// read before the same call wrote it, so nothing needs clearing between calls.
// ---------------------------------------------------------------------------------------------
constexpr int64_t kScratchBytes = int64_t(64) << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

static uint8_t *scratch_address() {
  static std::mutex mu;
  static std::map<int, uint8_t *> addr;  // device -> address of its copy of `scratch`
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) raise(PDLP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  addr[dev] = static_cast<uint8_t *>(ptr);
  return addr[dev];
}

template <typename T>
void variable_strategy_noalloc(Solver<T> &s, int strategy, int tiebreak, const uint8_t *var_type, const double *x,
                               const double *y, const double *rc, int32_t *order, int32_t *count) {
  for (const void *q : {(const void *)var_type, (const void *)x, (const void *)y, (const void *)rc, (const void *)order})
    if (q && !on_device(q)) raise(PDLP_ERR_ARG, "pdlp_variable_strategy_noalloc takes device pointers only");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != s.device) raise(PDLP_ERR_ARG, "the handle's GPU must be the current device");
  ScratchWork w{scratch_address(), kScratchBytes};
  variable_strategy_in(s, w, strategy, tiebreak, var_type, x, y, rc, order, count);
}

template <typename T>
void lp_fixing(Solver<T> &s, const uint8_t *var_type, const double *x, const double *l, const double *u,
               const double *uniform, double *value) {
  if (!var_type || !x || !l || !u || !uniform || !value) raise(PDLP_ERR_ARG, "NULL argument to pdlp_lp_fixing");
  if (s.K != 1) raise(PDLP_ERR_ARG, "LP-based fixing takes a single-problem handle");
  const int n = s.n;
  if (!on_device(x) && !finite_host(x, n)) raise(PDLP_ERR_ARG, "x must be finite");
  for (const double *b : {l, u})
    if (!on_device(b))
      for (int j = 0; j < n; ++j)
        if (std::isnan(b[j])) raise(PDLP_ERR_ARG, "bounds must not be NaN");
  if (!on_device(uniform))
    for (int j = 0; j < n; ++j)
      if (!(uniform[j] > 0.0 && uniform[j] < 1.0)) raise(PDLP_ERR_ARG, "samples must lie in (0, 1)");
  if (n == 0) return;
  hipStream_t st = s.stream;
  Work w(s.mem, cache_of(s));
  const uint8_t *d_vt = device_input(w, var_type, n, st);
  const double *d_x = device_input(w, x, n, st), *d_l = device_input(w, l, n, st);
  const double *d_u = device_input(w, u, n, st), *d_s = device_input(w, uniform, n, st);
  double *d_out = on_device(value) ? value : w.get<double>(n);
  hipLaunchKernelGGL(k_lp_fixing, dim3(fix_grid(n)), dim3(kSortBlock), 0, st, n, d_x, d_l, d_u, d_vt, d_s, d_out);
  HIPCHK(hipGetLastError());
  if (d_out != value) HIPCHK(hipMemcpyAsync(value, d_out, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
}

}  // namespace fix
}  // namespace pdlp

extern "C" {

int pdlp_variable_strategy(pdlp_problem *p, int32_t strategy, int32_t tiebreak, const uint8_t *var_type,
                           const double *x, const double *y, const double *red_cost, int32_t *order,
                           int32_t *count) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    p->s.visit([&](auto &s) { pdlp::fix::variable_strategy(s, strategy, tiebreak, var_type, x, y, red_cost, order, count); });
  });
}

int pdlp_variable_strategy_noalloc(pdlp_problem *p, int32_t strategy, int32_t tiebreak, const uint8_t *var_type,
                                   const double *x, const double *y, const double *red_cost, int32_t *order,
                                   int32_t *count) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    p->s.visit([&](auto &s) {
      pdlp::fix::variable_strategy_noalloc(s, strategy, tiebreak, var_type, x, y, red_cost, order, count);
    });
  });
}

int pdlp_lp_fixing(pdlp_problem *p, const uint8_t *var_type, const double *x, const double *l, const double *u,
                   const double *uniform, double *value) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { p->s.visit([&](auto &s) { pdlp::fix::lp_fixing(s, var_type, x, l, u, uniform, value); }); });
}

}  // extern "C"
