// Host side of linear-constraint propagation and of the integer-aware branching rule: the
// propagation handle and the extern "C" entry points declared in include/pdlp_prop.h. Included at
// the end of pdlp.hip (it uses Arena, HostProblem, validate, HIPCHK and guarded from there).
#pragma once

#include <cmath>
#include <vector>

#include "../../include/pdlp_prop.h"
#include "prop_kernels.h"

struct pdlp_prop {
  pdlp::Arena mem;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  int32_t *rp = nullptr, *ci = nullptr;
  int32_t *long_rows = nullptr;  // rows of at least kLongRow entries (one wave each)
  int32_t nlong = 0;
  double *val = nullptr, *b = nullptr;
  uint8_t *sense = nullptr, *vt = nullptr;
  double *l = nullptr, *u = nullptr;  // the caller's bounds staged on the device
  pdlp::prop::Bounds *lu = nullptr, *lun = nullptr;  // current and next bounds, by column
  int32_t *flags = nullptr;       // device: moved, row infeasible, bound crossed
  int32_t *h_flags = nullptr;     // pinned host copy
  ~pdlp_prop() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (h_flags) (void)hipHostFree(h_flags);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace pdlp {
namespace prop {

static int prop_grid(int64_t n) {
  const int64_t g = (n + kPropBlock - 1) / kPropBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 16384));
}

static bool on_device_mem(const void *p) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

template <typename U>
U *upload_new(pdlp_prop &p, const std::vector<U> &v) {
  U *d = p.mem.alloc<U>((int64_t)v.size());
  if (!v.empty()) HIPCHK(hipMemcpyAsync(d, v.data(), sizeof(U) * v.size(), hipMemcpyHostToDevice, p.stream));
  return d;
}

}  // namespace prop
}  // namespace pdlp

extern "C" {

int pdlp_prop_create(pdlp_prop **out, int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                     const int32_t *col_idx, const double *val, const double *b, const char *sense,
                     const uint8_t *var_type, const pdlp_options *opt) {
  if (!out || (n > 0 && !var_type)) {
    pdlp::g_last_error = "bad argument to pdlp_prop_create";
    return PDLP_ERR_ARG;
  }
  *out = nullptr;
  return guarded([&] {
    using pdlp::raise;
    const pdlp_options o = resolve_options(opt);
    // validate as an LP with free columns (costs and bounds are not part of this handle)
    std::vector<double> zero((size_t)std::max(n, 0), 0.0), lo((size_t)std::max(n, 0), -HUGE_VAL),
        hi((size_t)std::max(n, 0), HUGE_VAL);
    pdlp::HostProblem H;
    fetch_host_problem(H, m, n, nnz, row_ptr, col_idx, val, zero.data(), b, sense, lo.data(), hi.data(), false);
    std::vector<uint8_t> vt(var_type, var_type + std::max(n, 0));
    for (uint8_t t : vt)
      if (t > 2) raise(PDLP_ERR_ARG, "var_type must be 0 (continuous), 1 (binary) or 2 (integer)");
    auto p = std::make_unique<pdlp_prop>();
    p->mem.limit = o.device_mem_limit;
    if (o.stream) {
      p->stream = (hipStream_t)o.stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
      p->own_stream = true;
    }
    HIPCHK(hipHostMalloc((void **)&p->h_flags, 3 * sizeof(int32_t), hipHostMallocDefault));
    p->m = m, p->n = n, p->nnz = nnz;
    p->rp = pdlp::prop::upload_new(*p, H.rp);
    std::vector<int32_t> lr;
    for (int32_t i = 0; i < m; ++i)
      if (H.rp[i + 1] - H.rp[i] >= pdlp::prop::kLongRow) lr.push_back(i);
    p->nlong = (int32_t)lr.size();
    p->long_rows = pdlp::prop::upload_new(*p, lr);
    p->ci = pdlp::prop::upload_new(*p, H.ci);
    p->val = pdlp::prop::upload_new(*p, H.val);
    p->b = pdlp::prop::upload_new(*p, H.b);
    std::vector<uint8_t> sn(H.sense.begin(), H.sense.end());
    p->sense = pdlp::prop::upload_new(*p, sn);
    p->vt = pdlp::prop::upload_new(*p, vt);
    for (double **q : {&p->l, &p->u}) *q = p->mem.alloc<double>(n);
    p->lu = p->mem.alloc<pdlp::prop::Bounds>(n);
    p->lun = p->mem.alloc<pdlp::prop::Bounds>(n);
    p->flags = p->mem.alloc<int32_t>(3);
    HIPCHK(hipStreamSynchronize(p->stream));
    *out = p.release();
  });
}

int pdlp_propagate(pdlp_prop *p, double *l, double *u, int32_t max_rounds, int32_t *rounds, int32_t *status) {
  if (!p || max_rounds < 1 || (p->n > 0 && (!l || !u))) {
    pdlp::g_last_error = "bad argument to pdlp_propagate";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    using namespace pdlp::prop;
    const int n = p->n, m = p->m;
    hipStream_t st = p->stream;
    const bool dev_l = n > 0 && on_device_mem(l), dev_u = n > 0 && on_device_mem(u);
    if (!dev_l)
      for (int j = 0; j < n; ++j)
        if (std::isnan(l[j])) pdlp::raise(PDLP_ERR_ARG, "bounds must not be NaN");
    if (!dev_u)
      for (int j = 0; j < n; ++j)
        if (std::isnan(u[j])) pdlp::raise(PDLP_ERR_ARG, "bounds must not be NaN");
    // device bounds are read and written in place; host bounds go through the staging arrays
    double *dl = dev_l ? l : p->l, *du = dev_u ? u : p->u;
    if (n > 0) {
      const size_t bytes = sizeof(double) * (size_t)n;
      if (!dev_l) HIPCHK(hipMemcpyAsync(p->l, l, bytes, hipMemcpyHostToDevice, st));
      if (!dev_u) HIPCHK(hipMemcpyAsync(p->u, u, bytes, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_prop_pack, dim3(prop_grid(n)), dim3(kPropBlock), 0, st, n, (const double *)dl,
                         (const double *)du, p->lu, p->lun);
    }
    int32_t r = 0, stat = PDLP_PROP_ROUND_LIMIT;
    while (r < max_rounds) {
      HIPCHK(hipMemsetAsync(p->flags, 0, 3 * sizeof(int32_t), st));
      if (m > 0)
        hipLaunchKernelGGL(k_prop_round, dim3(prop_grid(m)), dim3(kPropBlock), 0, st, m, (const int32_t *)p->rp,
                           (const int32_t *)p->ci, (const double *)p->val, (const double *)p->b,
                           (const uint8_t *)p->sense, (const uint8_t *)p->vt, (const Bounds *)p->lu, p->lun,
                           p->flags);
      if (p->nlong > 0)
        hipLaunchKernelGGL(k_prop_round_long, dim3(prop_grid((int64_t)p->nlong * 64)), dim3(kPropBlock), 0, st,
                           p->nlong, (const int32_t *)p->long_rows, (const int32_t *)p->rp, (const int32_t *)p->ci,
                           (const double *)p->val, (const double *)p->b, (const uint8_t *)p->sense,
                           (const uint8_t *)p->vt, (const Bounds *)p->lu, p->lun, p->flags);
      if (n > 0)
        hipLaunchKernelGGL(k_prop_finish, dim3(prop_grid(n)), dim3(kPropBlock), 0, st, n, p->lu,
                           (const Bounds *)p->lun, p->flags);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(p->h_flags, p->flags, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      ++r;
      if (p->h_flags[1] || p->h_flags[2]) {
        stat = PDLP_PROP_INFEASIBLE;
        break;
      }
      if (!p->h_flags[0]) {
        stat = PDLP_PROP_FIXPOINT;
        break;
      }
    }
    if (n > 0) {
      const size_t bytes = sizeof(double) * (size_t)n;
      hipLaunchKernelGGL(k_prop_unpack, dim3(prop_grid(n)), dim3(kPropBlock), 0, st, n, (const Bounds *)p->lu, dl,
                         du);
      HIPCHK(hipGetLastError());
      if (!dev_l) HIPCHK(hipMemcpyAsync(l, p->l, bytes, hipMemcpyDeviceToHost, st));
      if (!dev_u) HIPCHK(hipMemcpyAsync(u, p->u, bytes, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    if (rounds) *rounds = r;
    if (status) *status = stat;
  });
}

void pdlp_prop_destroy(pdlp_prop *p) { delete p; }

int pdlp_branching(double l, double u, double a, double c, double *lower, double *upper, int32_t *count) {
  if (!lower || !upper || !count || std::isnan(l) || std::isnan(u) || std::isnan(a) || std::isnan(c) || a < l ||
      a > u || a != std::floor(a)) {
    pdlp::g_last_error = "pdlp_branching needs l <= a <= u with an integral a";
    return PDLP_ERR_ARG;
  }
  int k = 0;
  auto put = [&](double lo, double hi) { lower[k] = lo, upper[k] = hi, ++k; };
  if (l < a && a < u) {
    // the fixing last (highest priority), the restriction in the objective direction before it
    if (c > 0.0) put(a + 1.0, u), put(l, a - 1.0);
    else put(l, a - 1.0), put(a + 1.0, u);
    put(a, a);
  } else if (a == l) {
    put(u, u), put(l, l);
  } else {
    put(l, l), put(u, u);
  }
  *count = k;
  return 0;
}

}  // extern "C"
