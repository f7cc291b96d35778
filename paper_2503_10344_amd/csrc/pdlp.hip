// libpdlp host runtime: problem set-up on the device, the solve loop (one captured hipGraph per
// evaluation interval), finalisation and the extern "C" boundary declared in include/pdlp.h.
//
// A handle holds K >= 1 LPs as one block-diagonal problem (pdlp_create: K = 1; pdlp_batch_create:
// K = k). Set-up runs once over the concatenation (scaling and transposition of a block-diagonal
// matrix act on each block independently); the per-instance scalars are segmented reductions.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pdlp.h"
#include "pdlp_kernels.h"
#include "snap_kernels.h"

namespace pdlp {

// ----------------------------------------------------------------------------------------------
// Errors
// ----------------------------------------------------------------------------------------------
thread_local std::string g_last_error;

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] static void raise(int code, const std::string &msg) { throw Error{code, msg}; }

#define HIPCHK(expr)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      (void)hipGetLastError();                                                                  \
      raise(e_ == hipErrorOutOfMemory ? PDLP_ERR_OOM : PDLP_ERR_HIP,                            \
            std::string(#expr) + ": " + hipGetErrorString(e_));                                 \
    }                                                                                           \
  } while (0)

static int grid_for(int64_t n, int per_thread = 1, int cap = 4096) {
  int64_t g = (n + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// ----------------------------------------------------------------------------------------------
// Device memory owned by a handle, with an optional cap (forced out-of-memory tests use it).
// ----------------------------------------------------------------------------------------------
struct Arena {
  int64_t limit = 0, used = 0;
  std::vector<std::pair<void *, int64_t>> blocks;
  template <typename U>
  U *alloc(int64_t count) {
    int64_t bytes = std::max<int64_t>(count, 1) * (int64_t)sizeof(U);
    bytes = (bytes + 255) & ~int64_t(255);
    if (limit > 0 && used + bytes > limit)
      raise(PDLP_ERR_OOM, "device_mem_limit of " + std::to_string(limit) + " bytes exceeded");
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      raise(PDLP_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    used += bytes;
    blocks.push_back({p, bytes});
    return static_cast<U *>(p);
  }
  void release(void *p) {
    for (size_t i = 0; i < blocks.size(); ++i)
      if (blocks[i].first == p) {
        (void)hipFree(p);
        used -= blocks[i].second;
        blocks.erase(blocks.begin() + (long)i);
        return;
      }
  }
  void reset() {
    for (auto &b : blocks) (void)hipFree(b.first);
    blocks.clear();
    used = 0;
  }
  ~Arena() { reset(); }
};

// ----------------------------------------------------------------------------------------------
// Host copy of one LP (eq. (1) with row senses) and its validation.
// ----------------------------------------------------------------------------------------------
struct HostProblem {
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> val, c, b, l, u;
  std::vector<uint8_t> sense;
};

static void validate(const HostProblem &P) {
  if (P.m < 0 || P.n < 0) raise(PDLP_ERR_ARG, "negative dimension");
  if (P.nnz < 0 || P.nnz >= (int64_t)INT32_MAX) raise(PDLP_ERR_ARG, "nnz out of range");
  if (P.rp[0] != 0 || P.rp[P.m] != P.nnz) raise(PDLP_ERR_CSR, "row_ptr[0] must be 0 and row_ptr[m] == nnz");
  for (int32_t i = 0; i < P.m; ++i) {
    const int32_t a = P.rp[i], e = P.rp[i + 1];
    if (e < a) raise(PDLP_ERR_CSR, "row_ptr decreases at row " + std::to_string(i));
    for (int32_t k = a; k < e; ++k) {
      const int32_t j = P.ci[k];
      if (j < 0 || j >= P.n) raise(PDLP_ERR_CSR, "column index out of range in row " + std::to_string(i));
      if (k > a && j <= P.ci[k - 1])
        raise(PDLP_ERR_CSR, "column indices not strictly increasing (duplicate or unsorted) in row " +
                                std::to_string(i));
    }
    const uint8_t s = P.sense[i];
    if (s != 'L' && s != 'G' && s != 'E') raise(PDLP_ERR_ARG, "row sense must be 'L', 'G' or 'E'");
    if (!std::isfinite(P.b[i])) raise(PDLP_ERR_ARG, "b must be finite");
  }
  for (int64_t k = 0; k < P.nnz; ++k)
    if (!std::isfinite(P.val[k])) raise(PDLP_ERR_ARG, "matrix values must be finite");
  for (int32_t j = 0; j < P.n; ++j) {
    if (!std::isfinite(P.c[j])) raise(PDLP_ERR_ARG, "c must be finite");
    if (std::isnan(P.l[j]) || std::isnan(P.u[j])) raise(PDLP_ERR_ARG, "bounds must not be NaN");
    if (P.l[j] > P.u[j]) raise(PDLP_ERR_ARG, "l > u at column " + std::to_string(j));
    if (P.l[j] == INFINITY || P.u[j] == -INFINITY) raise(PDLP_ERR_ARG, "l = +inf or u = -inf");
  }
}

// Length class of a row (see chunk_rows): 0 for len <= 3, else floor(log2 len) - 1, at most 6.
static int length_class(int64_t len) {
  if (len <= 3) return 0;
  const int c = 62 - __builtin_clzll((unsigned long long)len);
  return c < 6 ? c : 6;
}

// Chunks of rows [r0, r1) (rows sorted by descending class): runs of consecutive rows of one class
// with at most `cap` nonzeros (a longer row alone) and at most four wave passes. Chunk boundaries
// are appended to `rows`, classes to `cls`. An empty range yields one empty chunk so that every
// instance owns at least one.
static void build_chunks(const int32_t *rp, int32_t r0, int32_t r1, int cap, std::vector<int32_t> &rows,
                         std::vector<int8_t> &cls) {
  if (r1 == r0) {
    rows.push_back(r1);
    cls.push_back(0);
    return;
  }
  int32_t start = r0;
  int c_start = length_class((int64_t)rp[r0 + 1] - rp[r0]);
  int64_t acc = 0;
  for (int32_t i = r0; i < r1; ++i) {
    const int64_t len = (int64_t)rp[i + 1] - rp[i];
    const int c = length_class(len);
    const int max_rows = (kWave >> c_start) * 4;
    if (i > start && (c != c_start || acc + len > cap || i - start >= max_rows)) {
      rows.push_back(i);
      cls.push_back((int8_t)c_start);
      start = i, c_start = c, acc = 0;
    }
    acc += len;
  }
  rows.push_back(r1);
  cls.push_back((int8_t)c_start);
}

// Stable order of the items [lo, hi) by descending length (so also by descending length class, and
// rows of similar length sit together for the column-panel blocks); out receives old indices.
static void class_order(const std::vector<int64_t> &len, int32_t lo, int32_t hi, std::vector<int32_t> &out) {
  std::vector<int32_t> idx;
  idx.reserve((size_t)(hi - lo));
  for (int32_t i = lo; i < hi; ++i) idx.push_back(i);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int32_t a, int32_t b) { return len[(size_t)(a - lo)] > len[(size_t)(b - lo)]; });
  out.insert(out.end(), idx.begin(), idx.end());
}

// Column-panel layout of the long rows (host side; see Panels in pdlp_internal.h).
constexpr int kPanelDefaultMinRow = 64;  // rows at least this long are summed by column panels
// target entries per (row block, panel) work group: on the 500k x 1M LP 8,192 / 16,384 / 20,480 /
// 24,576 / 28,672 / 32,768 gave k_panel 77.7 / 64.9 / 60.1 / 60.3 / 61.8 / 65.3 us
constexpr int kPanelEntries = 24576;
constexpr int kPanelMaxRows = 4096;      // rows per row block at most
constexpr int kPanelMaxPanels = 256;     // instances with more x panels keep the chunk engine
struct PanelHost {
  std::vector<int32_t> wg_rb, wg_p, rb_inst, rb_lrow0, rb_R, rb_G, src;
  std::vector<int64_t> wg_ebase, wg_obase;
  std::vector<uint16_t> off, col;
  void append(const PanelHost &o) {
    auto cat = [](auto &a, const auto &b) { a.insert(a.end(), b.begin(), b.end()); };
    cat(wg_rb, o.wg_rb), cat(wg_p, o.wg_p), cat(rb_inst, o.rb_inst), cat(rb_lrow0, o.rb_lrow0);
    cat(rb_R, o.rb_R), cat(rb_G, o.rb_G), cat(src, o.src), cat(wg_ebase, o.wg_ebase), cat(wg_obase, o.wg_obase);
    cat(off, o.off), cat(col, o.col);
  }
};

// Long rows of one instance (rows [r0, r0 + R) in internal order, columns [c0, c0 + nq)) cut into
// row blocks and panels. ci: internal column of each entry. src receives the CSR position of every
// entry of the layout (its value is gathered on the device). Returns false when a work group would
// need offsets beyond 16 bits (the instance then keeps the chunk engine for all rows).
static bool build_panels(const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, int q, int32_t r0,
                         int32_t R, int32_t c0, int32_t nq, PanelHost &H) {
  const int P = (nq + kPanelW - 1) / kPanelW;
  const int64_t target = (int64_t)kPanelEntries * P;
  const int64_t e0 = (int64_t)H.col.size(), o0 = (int64_t)H.off.size();
  const int rb0 = (int)H.rb_R.size();
  PanelHost out;
  int32_t r = 0;
  std::vector<int32_t> cnt;
  while (r < R) {
    int32_t e = r;
    int64_t acc = 0;
    while (e < R && (e == r || (acc + (rp[r0 + e + 1] - rp[r0 + e]) <= target && e - r < kPanelMaxRows))) {
      acc += rp[r0 + e + 1] - rp[r0 + e];
      ++e;
    }
    for (;;) {  // shrink the block until every (block, panel) holds fewer than 2^16 entries
      const int32_t nr = e - r;
      cnt.assign((size_t)P * (nr + 1), 0);
      for (int32_t i = 0; i < nr; ++i)
        for (int32_t k = rp[r0 + r + i]; k < rp[r0 + r + i + 1]; ++k) cnt[(size_t)((ci[k] - c0) / kPanelW) * (nr + 1) + i + 1]++;
      int64_t worst = 0;
      for (int p = 0; p < P; ++p) {
        int64_t t = 0;
        for (int32_t i = 0; i <= nr; ++i) t += cnt[(size_t)p * (nr + 1) + i];
        worst = std::max(worst, t);
      }
      if (worst < 65536) break;
      if (nr == 1) return false;
      e = r + nr / 2;
    }
    const int32_t nr = e - r;
    const int rb = rb0 + (int)out.rb_R.size();
    int64_t bnnz = (int64_t)rp[r0 + e] - rp[r0 + r];
    const double seg = (double)bnnz / nr / P / 4.0;  // entries per lane and panel with G lanes a row
    int G = 1;
    while (G < 64 && 2.0 * G <= seg) G *= 2;
    out.rb_inst.push_back(q), out.rb_lrow0.push_back(r), out.rb_R.push_back(nr), out.rb_G.push_back(G);
    for (int p = 0; p < P; ++p) {
      out.wg_rb.push_back(rb), out.wg_p.push_back(p);
      out.wg_ebase.push_back(e0 + (int64_t)out.col.size());
      out.wg_obase.push_back(o0 + (int64_t)out.off.size());
      int64_t run = 0;
      out.off.push_back(0);
      for (int32_t i = 0; i < nr; ++i) {
        for (int32_t k = rp[r0 + r + i]; k < rp[r0 + r + i + 1]; ++k) {
          const int32_t lc = ci[k] - c0;
          if (lc / kPanelW != p) continue;
          out.col.push_back((uint16_t)(lc - p * kPanelW));
          out.src.push_back(k);
          ++run;
        }
        out.off.push_back((uint16_t)run);
      }
    }
    r = e;
  }
  H.append(out);
  return true;
}

// Column-block layout of A' (host side; see ColBlocks in pdlp_internal.h).
struct ColBlockHost {
  std::vector<int32_t> wg_inst, wg_blk, wg_g0, gstart, ebase, src, wg_t, tebase, trow, tsrc;
  std::vector<uint32_t> desc, tdesc;
  std::vector<uint16_t> row;
};
// Auto mode: an instance takes column blocks when no column is longer than kCbAutoMaxCol and the
// handle holds at least kCbAutoNnz nonzeros in all. A work group owns 4,096 columns, so an instance
// alone fills the GPU only when it is large; in a batch the instances' work groups fill it together
// (256 LPs of 1k-50k rows: makespan 1.38 -> 0.92 s, while the same LPs one by one take 4.2 s without
// and 5.1 s with column blocks).
constexpr int64_t kCbAutoNnz = int64_t(1) << 20;
constexpr int kCbAutoMaxCol = 64;
constexpr double kCbDenseShare = 0.9;              // dense panels: the shortest prefix holding this share
constexpr int kRbMaxPanels = 8;  // row blocks of A x: instances with at most this many x panels

// Runs of one work group (column lc, first entry, length), sorted by length (longest first), dealt
// to 64-lane groups: descriptors, the group's first slot (of 64 entries), and per slot and lane the
// entry's index into crow / csrc (-1 past a run's end).
struct CbRun {
  int32_t lc, start, len;
};
template <typename Emit>
static void cb_groups(std::vector<CbRun> &runs, std::vector<uint32_t> &desc, std::vector<int32_t> &ebase,
                      int64_t &slots, Emit &&emit) {
  std::stable_sort(runs.begin(), runs.end(), [](const CbRun &a, const CbRun &c) { return a.len > c.len; });
  for (size_t g0 = 0; g0 < runs.size(); g0 += kWave) {
    const size_t gn = std::min<size_t>(kWave, runs.size() - g0);
    const int32_t glen = runs[g0].len;
    ebase.push_back((int32_t)slots);
    for (size_t l = 0; l < (size_t)kWave; ++l)
      desc.push_back(l < gn ? ((uint32_t)runs[g0 + l].len << 16) | (uint32_t)runs[g0 + l].lc : 0u);
    for (int32_t t = 0; t < glen; ++t)
      for (size_t l = 0; l < (size_t)kWave; ++l)
        emit(l < gn && t < runs[g0 + l].len ? runs[g0 + l].start + t : -1);
    slots += glen;
  }
}

// Line blocks of instance q: its nl lines (columns of A for A'y, rows of A for A x), line l's
// entries given in position order (lp: [nl + 1] offsets; lpos: position within the instance, i.e.
// row for a column, column for a row; lsrc: CSR position), over npos positions. Work groups of
// kCbCols lines, dense position panels of kCbRows and the tail, as the kernel reads them (layout in
// ColBlocks; "column" there is the line, "row" the position). src / tsrc receive the CSR position
// of every entry (-1: padding). Returns false (H unchanged) when a work group would have more than
// kCbMaxGroups groups of runs in its panels or a slot count leaves the int32 range.
static bool build_line_blocks(const std::vector<int32_t> &lp, const std::vector<int32_t> &lpos,
                              const std::vector<int32_t> &lsrc, int q, int32_t nl, int32_t npos, ColBlockHost &H,
                              int32_t *ndense) {
  const int64_t zq = lp[(size_t)nl];
  const int np = (npos + kCbRows - 1) / kCbRows, nb = (nl + kCbCols - 1) / kCbCols;
  // dense panels: the shortest prefix of panels holding kCbDenseShare of the entries
  int nd = 0;
  {
    std::vector<int64_t> per((size_t)std::max(np, 1), 0);
    for (int64_t k = 0; k < zq; ++k) per[(size_t)(lpos[k] / kCbRows)] += 1;
    int64_t acc = 0;
    while (nd < np && (double)acc < kCbDenseShare * (double)zq) acc += per[(size_t)nd++];
  }
  std::vector<int32_t> cur(lp.begin(), lp.end() - 1);  // next entry of each line
  ColBlockHost out;
  int64_t slots = (int64_t)H.row.size() / kWave;     // panel entry slots (of 64) before this instance
  int64_t tslots = (int64_t)H.trow.size() / kWave;   // tail entry slots before this instance
  const int64_t g_base = (int64_t)H.ebase.size(), t_base = (int64_t)H.tebase.size();
  std::vector<CbRun> runs;
  for (int b = 0; b < nb; ++b) {
    out.wg_inst.push_back(q), out.wg_blk.push_back(b);
    out.wg_g0.push_back((int32_t)(H.gstart.size() + out.gstart.size()));
    out.wg_t.push_back((int32_t)(t_base + (int64_t)out.tebase.size()));
    const int64_t wg_first = g_base + (int64_t)out.ebase.size();
    const int32_t jb = b * kCbCols, jn = std::min(kCbCols, nl - jb);
    for (int p = 0; p < nd; ++p) {
      out.gstart.push_back((int32_t)(g_base + (int64_t)out.ebase.size()));
      const int32_t pend = (p + 1) * kCbRows;
      runs.clear();
      for (int32_t lc = 0; lc < jn; ++lc) {
        const int32_t j = jb + lc;
        int32_t len = 0;
        while (cur[j] + len < lp[j + 1] && lpos[cur[j] + len] < pend) ++len;
        if (len > 0) runs.push_back({lc, cur[j], len});
        cur[j] += len;
      }
      cb_groups(runs, out.desc, out.ebase, slots, [&](int32_t k) {
        out.row.push_back(k >= 0 ? (uint16_t)(lpos[k] - p * kCbRows) : (uint16_t)0);
        out.src.push_back(k >= 0 ? lsrc[k] : -1);
      });
    }
    out.gstart.push_back((int32_t)(g_base + (int64_t)out.ebase.size()));
    runs.clear();
    for (int32_t lc = 0; lc < jn; ++lc) {
      const int32_t j = jb + lc;
      if (cur[j] < lp[j + 1]) runs.push_back({lc, cur[j], lp[j + 1] - cur[j]});
      cur[j] = lp[j + 1];
    }
    cb_groups(runs, out.tdesc, out.tebase, tslots, [&](int32_t k) {
      out.trow.push_back(k >= 0 ? lpos[k] : 0);
      out.tsrc.push_back(k >= 0 ? lsrc[k] : -1);
    });
    if (g_base + (int64_t)out.ebase.size() - wg_first > kCbMaxGroups || slots >= INT32_MAX / kWave ||
        tslots >= INT32_MAX / kWave)
      return false;
  }
  auto cat = [](auto &a, const auto &bb) { a.insert(a.end(), bb.begin(), bb.end()); };
  *ndense = nd;
  cat(H.wg_inst, out.wg_inst), cat(H.wg_blk, out.wg_blk), cat(H.wg_g0, out.wg_g0), cat(H.gstart, out.gstart);
  cat(H.ebase, out.ebase), cat(H.desc, out.desc), cat(H.row, out.row), cat(H.src, out.src);
  cat(H.wg_t, out.wg_t), cat(H.tebase, out.tebase), cat(H.tdesc, out.tdesc), cat(H.trow, out.trow);
  cat(H.tsrc, out.tsrc);
  return true;
}

// Columns of instance q (rows [r0, r0 + mq), columns [c0, c0 + nq); rp / ci: A in CSR, internal
// numbering): each column's entries in row order.
static bool build_col_blocks(const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, int q, int32_t r0,
                             int32_t mq, int32_t c0, int32_t nq, ColBlockHost &H, int32_t *ndense) {
  const int64_t z0 = rp[r0], zq = (int64_t)rp[r0 + mq] - z0;
  std::vector<int32_t> cp((size_t)nq + 1, 0), crow((size_t)zq), csrc((size_t)zq);
  for (int64_t k = z0; k < z0 + zq; ++k) cp[(size_t)(ci[k] - c0) + 1]++;
  for (int32_t j = 0; j < nq; ++j) cp[j + 1] += cp[j];
  std::vector<int32_t> fill(cp.begin(), cp.end() - 1);
  for (int32_t i = 0; i < mq; ++i)
    for (int32_t k = rp[r0 + i]; k < rp[r0 + i + 1]; ++k) {
      const int32_t j = ci[k] - c0;
      crow[fill[j]] = i, csrc[fill[j]] = k, ++fill[j];
    }
  return build_line_blocks(cp, crow, csrc, q, nq, mq, H, ndense);
}

// Rows of instance q: each row's entries in column order.
static bool build_row_blocks(const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, int q, int32_t r0,
                             int32_t mq, int32_t c0, int32_t nq, ColBlockHost &H, int32_t *ndense) {
  const int64_t z0 = rp[r0], zq = (int64_t)rp[r0 + mq] - z0;
  std::vector<int32_t> lp((size_t)mq + 1, 0), pos((size_t)zq), src((size_t)zq);
  std::vector<std::pair<int32_t, int32_t>> row;
  for (int32_t i = 0; i < mq; ++i) {
    row.clear();
    for (int32_t k = rp[r0 + i]; k < rp[r0 + i + 1]; ++k) row.push_back({ci[k] - c0, k});
    std::sort(row.begin(), row.end());
    const int64_t b = rp[r0 + i] - z0;
    for (size_t t = 0; t < row.size(); ++t) pos[(size_t)b + t] = row[t].first, src[(size_t)b + t] = row[t].second;
    lp[(size_t)i + 1] = (int32_t)(b + (int64_t)row.size());
  }
  return build_line_blocks(lp, pos, src, q, mq, nq, H, ndense);
}

static const int kChunkCandidates[] = {512, 1024, 2048, 4096};
// Smallest weight (nonzeros + rows) worth a work block of its own. Timed on MI355X: 1024 beats
// 2048 on small LPs (a 2k x 5k set cover solves in 13.7 instead of 16.2 ms, more blocks in flight)
// and matches it on the 256-LP batch; 512 makes the batch 20 % slower (per-block overhead).
static const int64_t kMinBlockWeight = 1024;
constexpr int kMaxResumes = 6;  // FP64 re-checks that may send an instance back into the loop

// Autotune cache: matrix signature -> chosen chunk size.
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune_cache;

// ----------------------------------------------------------------------------------------------
// Solver for K instances
// ----------------------------------------------------------------------------------------------
template <typename T>
struct Solver {
  pdlp_options opt{};
  int device = 0;  // the GPU that was current at create
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Arena mem;
  int32_t K = 1, m = 0, n = 0, nnz = 0;
  // instance layout (host)
  std::vector<int32_t> h_row0, h_col0, h_nnz0, h_a_chunk0, h_t_chunk0, h_ab0, h_tb0, h_ev0;
  std::vector<int32_t> h_arp, h_trp;
  std::string sig;
  // instance layout (device)
  int32_t *d_row0 = nullptr, *d_col0 = nullptr, *d_nnz0 = nullptr, *d_a_chunk0 = nullptr, *d_t_chunk0 = nullptr;
  int32_t *d_ab0 = nullptr, *d_ab_inst = nullptr, *d_tb0 = nullptr, *d_tb_inst = nullptr;
  int32_t *d_ev0 = nullptr, *d_ev_inst = nullptr;
  int32_t *d_a_bchunk = nullptr, *d_t_bchunk = nullptr;  // first chunk of each work block
  int ab_blocks = 1, tb_blocks = 1, ev_blocks = 1;
  int work_blocks = 16384;  // most work blocks per side of one instance
  // matrix
  int32_t *a_rp = nullptr, *a_ci = nullptr, *t_rp = nullptr, *t_ci = nullptr, *perm = nullptr;
  int32_t *a_chunk_row = nullptr, *t_chunk_row = nullptr;
  int8_t *a_chunk_cls = nullptr, *t_chunk_cls = nullptr;
  double *a_v64 = nullptr, *t_v64 = nullptr;
  T *a_v = nullptr, *t_v = nullptr;
  int chunk_nnz = 2048, a_nchunks = 0, t_nchunks = 0;
  // internal <-> external numbering (rows and columns sorted by length class per instance)
  std::vector<int32_t> h_perm_r, h_perm_c, h_inv_r, h_inv_c, h_nnz_map;
  int32_t *d_perm_r = nullptr, *d_perm_c = nullptr, *d_inv_r = nullptr, *d_inv_c = nullptr;
  // data
  uint8_t *sense = nullptr;
  double *Dr = nullptr, *Dc = nullptr, *c64 = nullptr, *b64 = nullptr, *l64 = nullptr, *u64 = nullptr;
  T *cT = nullptr, *bT = nullptr, *lT = nullptr, *uT = nullptr;
  // iterates
  T *xs[2] = {nullptr, nullptr}, *ys[2] = {nullptr, nullptr}, *axs[2] = {nullptr, nullptr};
  T *aty = nullptr, *axbar = nullptr, *atybar = nullptr;
  double *xbar = nullptr, *ybar = nullptr;  // running averages, FP64 in both precisions
  T *xa = nullptr, *ya = nullptr, *tmp_n = nullptr, *tmp_m = nullptr;
  // finalize / staging
  double *xd = nullptr, *yd = nullptr, *ax64 = nullptr, *aty64 = nullptr;
  double *x_out = nullptr, *y_out = nullptr, *rc_out = nullptr, *stage_n = nullptr, *stage_m = nullptr;
  double *x_ext = nullptr, *y_ext = nullptr, *rc_ext = nullptr;  // solution in the caller's numbering
  // reductions, state
  double *p_dual = nullptr, *p_primal = nullptr, *p_restart = nullptr, *p_eval = nullptr, *p_final = nullptr;
  double *d_red = nullptr;
  State *st = nullptr;
  int32_t *ndone = nullptr;
  std::vector<State> h_st;  // host mirror
  int32_t *h_flags = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<double> eta0, omega_default, nb, nc;
  hipGraphExec_t graph = nullptr;
  // kernel timing (opt.kernel_timing): two pools of start/stop events per attempt and kernel
  std::vector<hipEvent_t> tev[2];
  int64_t t_launches[5] = {0, 0, 0, 0, 0};
  double t_ms[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  Iter<T> P{};
  std::shared_ptr<void> fix_cache;  // workspace of the LP-based variable strategies, kept between calls
  // column-panel path of the long rows of A (FP32; PQ.nwg == 0: off). h_lr_*: see Layout.
  Panels<T> PQ{};
  double *part = nullptr;
  int64_t part_len = 0, pan_entries = 0;
  int32_t *pan_src = nullptr;  // CSR position of each layout entry (set-up only)
  std::vector<int32_t> h_lr_R, h_lr_P;
  std::vector<int64_t> h_lr_base;
  int32_t *d_lr_R = nullptr, *d_lr_P = nullptr;
  int64_t *d_lr_base = nullptr;
  // iteration layout of the A side (k_dual): per instance a skipped chunk over its long rows, the
  // chunks of its other rows and the long-row blocks. Equal to the product layout without panels.
  int32_t *ia_chunk_row = nullptr;
  int8_t *ia_chunk_cls = nullptr;
  int32_t *d_ia_ab0 = nullptr, *d_ia_ab_inst = nullptr, *d_ia_bchunk = nullptr;
  std::vector<int32_t> h_ia_ab0, h_ia_bc, h_t_bchunk;  // host copies of the last schedule built
  int ia_blocks = 1;
  // column blocks of A'y and row blocks of A x (FP32; nwg == 0: off). h_cb_n[q] / h_rb_n[q]: work
  // groups of instance q (0: the chunk engine); h_pb0 / h_db0: ranges of p_primal / p_dual pairs.
  struct LineBlocksSrc {  // CSR positions of a layout's entries (set-up only)
    int32_t *src = nullptr, *tsrc = nullptr;
    int64_t ne = 0, nte = 0;
  };
  ColBlocks<T> CQ{}, RQ{};
  LineBlocksSrc cb_src, rb_src;
  std::vector<int32_t> h_cb_n, h_cb_nd, h_rb_n, h_rb_nd, h_pb0, h_db0;
  int32_t *d_cb_n = nullptr, *d_rb_n = nullptr, *d_pb0 = nullptr, *d_db0 = nullptr;
  int4 *d_ia_desc = nullptr, *d_tb_desc = nullptr;  // start descriptors of k_dual / k_primal blocks
  int2 *d_tb_rows = nullptr;
  bool chunk_primal = true;  // some instance runs A'y by the chunk engine (k_primal)
  bool chunk_dual = true;    // some instance runs A x by k_dual
  // reference snapshots (restart points within snap.rel_tol; off while snap.K == 0)
  Snap snap{};
  bool solved = false;
  std::vector<pdlp_result> last;

  ~Solver() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto &pool : tev)
      for (auto e : pool) (void)hipEventDestroy(e);
    if (graph) (void)hipGraphExecDestroy(graph);
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
    if (h_flags) (void)hipHostFree(h_flags);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  template <typename U>
  void upload(U *dst, const U *src, int64_t count) {
    if (count > 0) HIPCHK(hipMemcpyAsync(dst, src, (size_t)count * sizeof(U), hipMemcpyHostToDevice, stream));
  }
  template <typename U>
  void download(U *dst, const U *src, int64_t count) {
    if (count > 0) HIPCHK(hipMemcpyAsync(dst, src, (size_t)count * sizeof(U), hipMemcpyDeviceToHost, stream));
  }
  template <typename U>
  U *alloc_upload(const std::vector<U> &v) {
    U *d = mem.alloc<U>((int64_t)v.size());
    upload(d, v.data(), (int64_t)v.size());
    return d;
  }
  void sync() { HIPCHK(hipStreamSynchronize(stream)); }

  // per-instance segmented reduction (kind 0 sum of squares, 1 max |v|) over segments s0
  std::vector<double> seg_reduce(int kind, const int32_t *d_s0, const double *v) {
    hipLaunchKernelGGL(k_seg_reduce, dim3(K), dim3(kBlock), 0, stream, kind, d_s0, v, d_red);
    HIPCHK(hipGetLastError());
    std::vector<double> r((size_t)K);
    download(r.data(), d_red, K);
    sync();
    return r;
  }

  // ---------------------------------------------------------------------------------------------
  void create(const std::vector<const HostProblem *> &Hs, const pdlp_options &o) {
    opt = o;
    HIPCHK(hipGetDevice(&device));
    if (o.work_blocks > 0) work_blocks = o.work_blocks;
    K = (int32_t)Hs.size();
    mem.limit = o.device_mem_limit;
    if (o.stream) {
      stream = (hipStream_t)o.stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
      own_stream = true;
    }
    HIPCHK(hipHostMalloc((void **)&h_flags, 2 * sizeof(int32_t), hipHostMallocDefault));
    for (auto &e : ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));

    // ---- concatenate ----
    h_row0.assign(1, 0), h_col0.assign(1, 0), h_nnz0.assign(1, 0);
    int64_t M = 0, N = 0, Z = 0;
    for (const HostProblem *H : Hs) {
      M += H->m, N += H->n, Z += H->nnz;
      if (M >= INT32_MAX || N >= INT32_MAX || Z >= INT32_MAX) raise(PDLP_ERR_ARG, "total size exceeds int32 range");
      h_row0.push_back((int32_t)M), h_col0.push_back((int32_t)N), h_nnz0.push_back((int32_t)Z);
    }
    m = (int32_t)M, n = (int32_t)N, nnz = (int32_t)Z;
    // concatenate, renumbering rows and columns of every instance by descending length class
    h_arp.assign((size_t)m + 1, 0);
    std::vector<int32_t> ci((size_t)nnz);
    std::vector<double> val((size_t)nnz), c((size_t)n), b((size_t)m), l((size_t)n), u((size_t)n);
    std::vector<uint8_t> sn((size_t)m);
    h_perm_r.clear(), h_perm_c.clear();
    h_inv_r.assign((size_t)m, 0), h_inv_c.assign((size_t)n, 0), h_nnz_map.assign((size_t)nnz, 0);
    for (int q = 0; q < K; ++q) {
      const HostProblem &H = *Hs[q];
      const int32_t r0 = h_row0[q], c0 = h_col0[q], z0 = h_nnz0[q];
      std::vector<int64_t> rlen((size_t)H.m), clen((size_t)H.n, 0);
      for (int32_t i = 0; i < H.m; ++i) rlen[i] = (int64_t)H.rp[i + 1] - H.rp[i];
      for (int64_t k = 0; k < H.nnz; ++k) clen[H.ci[k]] += 1;
      std::vector<int32_t> pr, pc;
      class_order(rlen, 0, H.m, pr);
      class_order(clen, 0, H.n, pc);
      for (int32_t i = 0; i < H.m; ++i) h_perm_r.push_back(r0 + pr[i]), h_inv_r[r0 + pr[i]] = r0 + i;
      for (int32_t j = 0; j < H.n; ++j) h_perm_c.push_back(c0 + pc[j]), h_inv_c[c0 + pc[j]] = c0 + j;
      int32_t z = z0;
      for (int32_t i = 0; i < H.m; ++i) {
        const int32_t old = pr[i];
        for (int32_t k = H.rp[old]; k < H.rp[old + 1]; ++k, ++z) {
          ci[z] = h_inv_c[c0 + H.ci[k]];
          val[z] = H.val[k];
          h_nnz_map[z0 + k] = z;
        }
        h_arp[r0 + i + 1] = z;
        b[r0 + i] = H.b[old];
        sn[r0 + i] = H.sense[old];
      }
      for (int32_t j = 0; j < H.n; ++j) {
        const int32_t old = pc[j];
        c[c0 + j] = H.c[old], l[c0 + j] = H.l[old], u[c0 + j] = H.u[old];
      }
    }
    // signature of the sparsity pattern (autotune cache key)
    {
      uint64_t h = 1469598103934665603ull;
      auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
      mix((uint64_t)K), mix((uint64_t)m), mix((uint64_t)n), mix((uint64_t)nnz);
      const int32_t step = std::max<int32_t>(1, m / 4096);
      for (int32_t i = 0; i <= m; i += step) mix((uint64_t)h_arp[i]);
      char buf[96];
      snprintf(buf, sizeof buf, "%d:%d:%d:%d:%016llx:%d", K, m, n, nnz, (unsigned long long)h, (int)sizeof(T));
      sig = buf;
    }

    // ---- column-panel layout of the long rows (FP32 iterations only) ----
    h_lr_R.assign((size_t)K, 0), h_lr_P.assign((size_t)K, 0), h_lr_base.assign((size_t)K, 0);
    PanelHost PH;
    if (sizeof(T) == sizeof(float) && o.panel_rows >= 0) {
      const int min_row = o.panel_rows > 0 ? o.panel_rows : kPanelDefaultMinRow;
      for (int q = 0; q < K; ++q) {
        const int32_t r0 = h_row0[q], r1 = h_row0[q + 1], c0 = h_col0[q], nq = h_col0[q + 1] - c0;
        int32_t R = 0;
        while (r0 + R < r1 && h_arp[r0 + R + 1] - h_arp[r0 + R] >= min_row) ++R;
        const int64_t long_nnz = (int64_t)h_arp[r0 + R] - h_arp[r0], inst_nnz = (int64_t)h_arp[r1] - h_arp[r0];
        const int P = (nq + kPanelW - 1) / kPanelW;
        // worth it when the long rows carry most of the instance's nonzeros
        if (R == 0 || nq == 0 || 2 * long_nnz < inst_nnz || P > kPanelMaxPanels) continue;
        if (!build_panels(h_arp, ci, q, r0, R, c0, nq, PH)) continue;
        h_lr_R[q] = R, h_lr_P[q] = P, h_lr_base[q] = part_len;
        part_len += (int64_t)P * R;
      }
    }

    // ---- column-block layout of A' (FP32 iterations only) ----
    h_cb_n.assign((size_t)K, 0), h_cb_nd.assign((size_t)K, 0);
    ColBlockHost CH;
    if (sizeof(T) == sizeof(float) && o.col_blocks >= 0) {
      for (int q = 0; q < K; ++q) {
        const int32_t r0 = h_row0[q], mq = h_row0[q + 1] - r0, c0 = h_col0[q], nq = h_col0[q + 1] - c0;
        if (mq == 0 || nq == 0 || (mq + kCbRows - 1) / kCbRows > kCbMaxPanels) continue;
        if (o.col_blocks == 0) {
          if ((int64_t)nnz < kCbAutoNnz) continue;
          int32_t longest = 0;
          {
            std::vector<int32_t> cl((size_t)nq, 0);
            for (int64_t k = h_arp[r0]; k < h_arp[r0 + mq]; ++k) longest = std::max(longest, ++cl[ci[k] - c0]);
          }
          if (longest > kCbAutoMaxCol) continue;
        }
        const size_t w_before = CH.wg_inst.size();
        if (!build_col_blocks(h_arp, ci, q, r0, mq, c0, nq, CH, &h_cb_nd[q])) continue;  // CH unchanged then
        h_cb_n[q] = (int32_t)(CH.wg_inst.size() - w_before);
      }
    }
    // ---- row blocks of A x: instances with column blocks, no long-row panels and few x panels ----
    h_rb_n.assign((size_t)K, 0), h_rb_nd.assign((size_t)K, 0);
    ColBlockHost RH;
    for (int q = 0; q < K; ++q) {
      const int32_t r0 = h_row0[q], mq = h_row0[q + 1] - r0, c0 = h_col0[q], nq = h_col0[q + 1] - c0;
      if (!h_cb_n[q] || h_lr_R[q] > 0 || (nq + kCbRows - 1) / kCbRows > kRbMaxPanels) continue;
      const size_t w_before = RH.wg_inst.size();
      if (!build_row_blocks(h_arp, ci, q, r0, mq, c0, nq, RH, &h_rb_nd[q])) continue;  // RH unchanged then
      h_rb_n[q] = (int32_t)(RH.wg_inst.size() - w_before);
    }

    const int64_t mm = std::max(m, 1), nn = std::max(n, 1);
    a_rp = alloc_upload(h_arp);
    a_ci = alloc_upload(ci);
    a_v64 = alloc_upload(val);
    sense = alloc_upload(sn);
    double *c0 = alloc_upload(c), *b0 = alloc_upload(b), *l0 = alloc_upload(l), *u0 = alloc_upload(u);
    d_row0 = alloc_upload(h_row0), d_col0 = alloc_upload(h_col0), d_nnz0 = alloc_upload(h_nnz0);
    d_perm_r = alloc_upload(h_perm_r), d_perm_c = alloc_upload(h_perm_c);
    d_inv_r = alloc_upload(h_inv_r), d_inv_c = alloc_upload(h_inv_c);
    t_rp = mem.alloc<int32_t>(n + 1);
    t_ci = mem.alloc<int32_t>(nnz);
    perm = mem.alloc<int32_t>(nnz);
    Dr = mem.alloc<double>(mm), Dc = mem.alloc<double>(nn);
    c64 = mem.alloc<double>(nn), l64 = mem.alloc<double>(nn), u64 = mem.alloc<double>(nn);
    b64 = mem.alloc<double>(mm);
    d_red = mem.alloc<double>(K);
    st = mem.alloc<State>(K);
    ndone = mem.alloc<int32_t>(1);
    h_st.resize((size_t)K);
    last.assign((size_t)K, pdlp_result{});
    ci.clear(), ci.shrink_to_fit(), val.clear(), val.shrink_to_fit();
    d_lr_R = alloc_upload(h_lr_R), d_lr_P = alloc_upload(h_lr_P), d_lr_base = alloc_upload(h_lr_base);
    if (!PH.wg_rb.empty()) {
      PQ.nwg = (int32_t)PH.wg_rb.size();
      PQ.wg_rb = alloc_upload(PH.wg_rb), PQ.wg_p = alloc_upload(PH.wg_p);
      PQ.wg_ebase = alloc_upload(PH.wg_ebase), PQ.wg_obase = alloc_upload(PH.wg_obase);
      PQ.rb_inst = alloc_upload(PH.rb_inst), PQ.rb_lrow0 = alloc_upload(PH.rb_lrow0);
      PQ.rb_R = alloc_upload(PH.rb_R), PQ.rb_G = alloc_upload(PH.rb_G);
      PQ.off = alloc_upload(PH.off), PQ.col = alloc_upload(PH.col);
      pan_src = alloc_upload(PH.src);
      pan_entries = (int64_t)PH.src.size();
      part = mem.alloc<double>(std::max<int64_t>(part_len, 1));
    }
    PH = PanelHost{};
    d_cb_n = alloc_upload(h_cb_n), d_rb_n = alloc_upload(h_rb_n);
    chunk_primal = false, chunk_dual = false;
    for (int q = 0; q < K; ++q) chunk_primal |= h_cb_n[q] == 0, chunk_dual |= h_rb_n[q] == 0;
    upload_line_blocks(CH, h_cb_nd, CQ, cb_src);
    upload_line_blocks(RH, h_rb_nd, RQ, rb_src);
    CH = ColBlockHost{}, RH = ColBlockHost{};

    // ---- transpose (counting sort; the per-column sort of source positions makes it deterministic)
    int32_t *row_of = mem.alloc<int32_t>(nnz);
    int32_t *cnt = mem.alloc<int32_t>(nn);
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)nn, stream));
    hipLaunchKernelGGL(k_expand_rows, dim3(grid_for((int64_t)m * kWave)), dim3(kBlock), 0, stream, m, a_rp, row_of);
    hipLaunchKernelGGL(k_histogram, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, nnz, a_ci, cnt);
    const int nsb = (int)std::max<int64_t>(1, ((int64_t)n + kScanItems - 1) / kScanItems);
    int32_t *bsum = mem.alloc<int32_t>(nsb);
    hipLaunchKernelGGL(k_scan_partial, dim3(nsb), dim3(kBlock), 0, stream, n, cnt, bsum);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(kBlock), 0, stream, nsb, bsum);
    hipLaunchKernelGGL(k_scan_final, dim3(nsb), dim3(kBlock), 0, stream, n, cnt, bsum, t_rp);
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)nn, stream));
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, nnz, a_ci, t_rp, cnt, perm);
    HIPCHK(hipGetLastError());
    h_trp.resize((size_t)n + 1);
    download(h_trp.data(), t_rp, n + 1);
    sync();
    std::vector<int32_t> big;
    std::vector<int64_t> scr_off;
    int64_t scr_total = 0;
    for (int32_t j = 0; j < n; ++j) {
      const int32_t len = h_trp[j + 1] - h_trp[j];
      if (len > 32) {
        big.push_back(j);
        int64_t Np = 1;
        while (Np < len) Np <<= 1;
        scr_off.push_back(scr_total);
        if (Np > kSortLds) scr_total += Np;
      }
    }
    hipLaunchKernelGGL(k_segsort_small, dim3(grid_for(n)), dim3(kBlock), 0, stream, n, t_rp, perm);
    if (!big.empty()) {
      int32_t *d_big = alloc_upload(big);
      int64_t *d_off = alloc_upload(scr_off);
      int32_t *scr = mem.alloc<int32_t>(std::max<int64_t>(scr_total, 1));
      for (size_t off = 0; off < big.size(); off += 65535) {
        const int cntb = (int)std::min<size_t>(65535, big.size() - off);
        hipLaunchKernelGGL(k_segsort_large, dim3(cntb), dim3(kBlock), 0, stream, d_big + off, t_rp, perm, scr,
                           d_off + off);
      }
      HIPCHK(hipGetLastError());
      sync();
      mem.release(d_big), mem.release(d_off), mem.release(scr);
    }

    // ---- scaling: Ruiz passes then one Pock-Chambolle pass (FP64) ----
    double *rho = mem.alloc<double>(mm), *kap = mem.alloc<double>(nn);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(m)), dim3(kBlock), 0, stream, (int64_t)m, Dr, 1.0);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, stream, (int64_t)n, Dc, 1.0);
    auto pass = [&](bool sum) {
      auto rk = sum ? k_row_norm<true> : k_row_norm<false>;
      hipLaunchKernelGGL(rk, dim3(grid_for((int64_t)m * kWave)), dim3(kBlock), 0, stream, m, (const int32_t *)a_rp,
                         (const int32_t *)nullptr, (const double *)a_v64, rho);
      hipLaunchKernelGGL(rk, dim3(grid_for((int64_t)n * kWave)), dim3(kBlock), 0, stream, n, (const int32_t *)t_rp,
                         (const int32_t *)perm, (const double *)a_v64, kap);
      hipLaunchKernelGGL(k_apply_scale, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, nnz, (const int32_t *)row_of,
                         (const int32_t *)a_ci, a_v64, (const double *)rho, (const double *)kap);
      hipLaunchKernelGGL(k_div_inplace, dim3(grid_for(m)), dim3(kBlock), 0, stream, m, Dr, (const double *)rho);
      hipLaunchKernelGGL(k_div_inplace, dim3(grid_for(n)), dim3(kBlock), 0, stream, n, Dc, (const double *)kap);
    };
    for (int it = 0; it < o.ruiz_iters; ++it) pass(false);
    if (o.pock_chambolle) pass(true);
    HIPCHK(hipGetLastError());
    t_v64 = mem.alloc<double>(nnz);
    hipLaunchKernelGGL(k_gather_t<double>, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, nnz, (const int32_t *)perm,
                       (const int32_t *)row_of, (const double *)a_v64, t_ci, t_v64);
    cT = mem.alloc<T>(nn), lT = mem.alloc<T>(nn), uT = mem.alloc<T>(nn), bT = mem.alloc<T>(mm);
    hipLaunchKernelGGL(k_scale_vectors<T>, dim3(grid_for(std::max(m, n))), dim3(kBlock), 0, stream, m, n,
                       (const double *)c0, (const double *)l0, (const double *)u0, (const double *)b0,
                       (const double *)Dr, (const double *)Dc, c64, l64, u64, b64, cT, lT, uT, bT);
    HIPCHK(hipGetLastError());
    // ---- per-instance scalars ----
    nb = seg_reduce(0, d_row0, b0), nc = seg_reduce(0, d_col0, c0);
    const std::vector<double> ncs = seg_reduce(0, d_col0, c64), nbs = seg_reduce(0, d_row0, b64);
    const std::vector<double> amax = seg_reduce(1, d_nnz0, a_v64);
    eta0.resize((size_t)K), omega_default.resize((size_t)K);
    for (int q = 0; q < K; ++q) {
      nb[q] = std::sqrt(nb[q]), nc[q] = std::sqrt(nc[q]);
      const double a = std::sqrt(ncs[q]), bb = std::sqrt(nbs[q]);
      omega_default[q] = (a > 1e-10 && bb > 1e-10) ? a / bb : 1.0;
      eta0[q] = amax[q] > 0.0 ? 1.0 / amax[q] : 1.0;
    }
    mem.release(c0), mem.release(b0), mem.release(l0), mem.release(u0);
    mem.release(rho), mem.release(kap), mem.release(cnt), mem.release(bsum), mem.release(row_of);

    // iteration-precision copies of the matrix
    if (sizeof(T) == sizeof(double)) {
      a_v = reinterpret_cast<T *>(a_v64);
      t_v = reinterpret_cast<T *>(t_v64);
    } else {
      a_v = mem.alloc<T>(nnz), t_v = mem.alloc<T>(nnz);
      hipLaunchKernelGGL(k_convert<T>, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, (int64_t)nnz,
                         (const double *)a_v64, a_v);
      hipLaunchKernelGGL(k_convert<T>, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, (int64_t)nnz,
                         (const double *)t_v64, t_v);
    }
    if (PQ.nwg > 0) {  // values of the panel layout, gathered from the iteration-precision matrix
      T *pv = mem.alloc<T>(std::max<int64_t>(pan_entries, 1));
      hipLaunchKernelGGL(k_gather_t<T>, dim3(grid_for(pan_entries)), dim3(kBlock), 0, stream, (int)pan_entries,
                         (const int32_t *)pan_src, (const int32_t *)nullptr, (const T *)a_v, (int32_t *)nullptr, pv);
      HIPCHK(hipGetLastError());
      PQ.val = pv;
      sync();
      mem.release(pan_src);
      pan_src = nullptr;
    }
    gather_line_values(CQ, cb_src);
    gather_line_values(RQ, rb_src);

    // iterates and staging
    for (int q = 0; q < 2; ++q) xs[q] = mem.alloc<T>(nn), ys[q] = mem.alloc<T>(mm), axs[q] = mem.alloc<T>(mm);
    aty = mem.alloc<T>(nn), xbar = mem.alloc<double>(nn), atybar = mem.alloc<T>(nn), xa = mem.alloc<T>(nn);
    ybar = mem.alloc<double>(mm), axbar = mem.alloc<T>(mm), ya = mem.alloc<T>(mm);
    tmp_n = mem.alloc<T>(nn), tmp_m = mem.alloc<T>(mm);
    xd = mem.alloc<double>(nn), yd = mem.alloc<double>(mm), ax64 = mem.alloc<double>(mm), aty64 = mem.alloc<double>(nn);
    x_out = mem.alloc<double>(nn), y_out = mem.alloc<double>(mm), rc_out = mem.alloc<double>(nn);
    stage_n = mem.alloc<double>(nn), stage_m = mem.alloc<double>(mm);
    x_ext = mem.alloc<double>(nn), y_ext = mem.alloc<double>(mm), rc_ext = mem.alloc<double>(nn);
    for (int q = 0; q < 2; ++q) {
      HIPCHK(hipMemsetAsync(xs[q], 0, sizeof(T) * (size_t)nn, stream));
      HIPCHK(hipMemsetAsync(ys[q], 0, sizeof(T) * (size_t)mm, stream));
      HIPCHK(hipMemsetAsync(axs[q], 0, sizeof(T) * (size_t)mm, stream));
    }
    for (T *p : {aty, atybar, xa, tmp_n}) HIPCHK(hipMemsetAsync(p, 0, sizeof(T) * (size_t)nn, stream));
    for (T *p : {axbar, ya, tmp_m}) HIPCHK(hipMemsetAsync(p, 0, sizeof(T) * (size_t)mm, stream));
    HIPCHK(hipMemsetAsync(xbar, 0, sizeof(double) * (size_t)nn, stream));
    HIPCHK(hipMemsetAsync(ybar, 0, sizeof(double) * (size_t)mm, stream));
    HIPCHK(hipMemsetAsync(st, 0, sizeof(State) * (size_t)K, stream));

    // ---- SpMV schedule, work blocks and evaluation blocks ----
    choose_schedule();
    std::vector<int32_t> ev_inst;
    h_ev0.assign(1, 0);
    for (int q = 0; q < K; ++q) {
      const int32_t mq = h_row0[q + 1] - h_row0[q], nq = h_col0[q + 1] - h_col0[q];
      const int ev = grid_for(std::max(mq, nq), kEvalSpan / kBlock, 2048);
      for (int r = 0; r < ev; ++r) ev_inst.push_back(q);
      h_ev0.push_back(h_ev0.back() + ev);
    }
    ev_blocks = h_ev0.back();
    d_ev_inst = alloc_upload(ev_inst);
    d_ev0 = alloc_upload(h_ev0);
    h_db0.assign(1, 0);
    for (int q = 0; q < K; ++q)
      h_db0.push_back(h_db0.back() + (h_rb_n[q] > 0 ? h_rb_n[q] : h_ia_ab0[q + 1] - h_ia_ab0[q]));
    d_db0 = alloc_upload(h_db0);
    p_dual = mem.alloc<double>((int64_t)std::max(h_db0.back(), 1) * 2);
    h_pb0.assign(1, 0);
    for (int q = 0; q < K; ++q) h_pb0.push_back(h_pb0.back() + (h_cb_n[q] > 0 ? h_cb_n[q] : h_tb0[q + 1] - h_tb0[q]));
    d_pb0 = alloc_upload(h_pb0);
    build_block_descriptors();
    p_primal = mem.alloc<double>(std::max(h_pb0.back(), 1));
    p_restart = mem.alloc<double>(ev_blocks);
    p_eval = mem.alloc<double>((int64_t)ev_blocks * kEvalNV);
    p_final = mem.alloc<double>((int64_t)ev_blocks * 5);
    set_params();
    sync();
  }

  // Start descriptors of the k_dual and k_primal blocks (Layout::ia_desc, tb_desc, tb_rows): the
  // same block -> work mapping as work_block and xcd_remap, resolved once here.
  void build_block_descriptors() {
    std::vector<int4> ia((size_t)std::max(ia_blocks, 1), make_int4(0, 0, 0, 0));
    for (int q = 0; q < K; ++q) {
      const int s0 = h_ia_ab0[q], nb = h_ia_ab0[q + 1] - s0;
      for (int t = 0; t < nb; ++t) {
        const int gb = s0 + xcd_remap(t, nb);
        ia[(size_t)(s0 + t)] = make_int4(q, h_ia_bc[2 * (size_t)gb], h_ia_bc[2 * (size_t)gb + 1], h_db0[q] + t);
      }
    }
    std::vector<int4> tb((size_t)std::max(tb_blocks, 1), make_int4(0, 0, 0, 0));
    std::vector<int2> tr((size_t)std::max(tb_blocks, 1), make_int2(0, 0));
    for (int q = 0; q < K; ++q) {
      const int s0 = h_tb0[q], nb = h_tb0[q + 1] - s0;
      const int64_t r0 = h_row0[q], mq = h_row0[q + 1] - r0;
      for (int t = 0; t < nb; ++t) {
        const int lb = xcd_remap(t, nb), gb = s0 + lb;
        // the share() split of the rows, as k_primal computed it
        tr[(size_t)(s0 + t)] = make_int2((int)(r0 + (lb * mq) / nb), (int)(r0 + ((lb + 1) * mq) / nb));
        tb[(size_t)(s0 + t)] = make_int4(q, h_t_bchunk[(size_t)gb], h_t_bchunk[(size_t)gb + 1], h_pb0[q] + t);
      }
    }
    d_ia_desc = alloc_upload(ia), d_tb_desc = alloc_upload(tb), d_tb_rows = alloc_upload(tr);
  }

  // Upload a line-block layout (column blocks or row blocks); the entries' CSR positions stay on
  // the device until gather_line_values fills the values.
  void upload_line_blocks(ColBlockHost &H, const std::vector<int32_t> &ndense, ColBlocks<T> &Q, LineBlocksSrc &S) {
    if (H.wg_inst.empty()) return;
    for (int l = 0; l < kWave; ++l) H.row.push_back(0), H.src.push_back(-1);  // the spare slot
    H.wg_t.push_back((int32_t)H.tebase.size());                                 // end of the last tail
    H.tebase.push_back((int32_t)(H.trow.size() / kWave));
    if (H.trow.empty()) H.trow.push_back(0), H.tsrc.push_back(-1);
    Q.nwg = (int32_t)H.wg_inst.size();
    Q.ndense = alloc_upload(ndense);
    Q.wg_inst = alloc_upload(H.wg_inst), Q.wg_blk = alloc_upload(H.wg_blk), Q.wg_g0 = alloc_upload(H.wg_g0);
    Q.gstart = alloc_upload(H.gstart), Q.desc = alloc_upload(H.desc), Q.ebase = alloc_upload(H.ebase);
    Q.row = alloc_upload(H.row);
    Q.wg_t = alloc_upload(H.wg_t), Q.tdesc = alloc_upload(H.tdesc), Q.tebase = alloc_upload(H.tebase);
    Q.trow = alloc_upload(H.trow);
    S.src = alloc_upload(H.src), S.ne = (int64_t)H.src.size();
    S.tsrc = alloc_upload(H.tsrc), S.nte = (int64_t)H.tsrc.size();
  }
  // The layout's values from the iteration-precision matrix (0 for padding entries).
  void gather_line_values(ColBlocks<T> &Q, LineBlocksSrc &S) {
    if (Q.nwg == 0) return;
    T *v = mem.alloc<T>(std::max<int64_t>(S.ne, 1)), *tv = mem.alloc<T>(std::max<int64_t>(S.nte, 1));
    hipLaunchKernelGGL(k_gather_or_zero<T>, dim3(grid_for(S.ne)), dim3(kBlock), 0, stream, S.ne,
                       (const int32_t *)S.src, (const T *)a_v, v);
    hipLaunchKernelGGL(k_gather_or_zero<T>, dim3(grid_for(S.nte)), dim3(kBlock), 0, stream, S.nte,
                       (const int32_t *)S.tsrc, (const T *)a_v, tv);
    HIPCHK(hipGetLastError());
    Q.val = v, Q.tval = tv;
    sync();
    mem.release(S.src), mem.release(S.tsrc);
    S = LineBlocksSrc{};
  }

  void set_params() {
    Layout &L = P.L;
    L.K = K;
    L.row0 = d_row0, L.col0 = d_col0, L.a_chunk0 = d_a_chunk0, L.t_chunk0 = d_t_chunk0;
    L.ab0 = d_ia_ab0, L.ab_inst = d_ia_ab_inst, L.tb0 = d_tb0, L.tb_inst = d_tb_inst;
    L.a_bchunk = d_ia_bchunk, L.t_bchunk = d_t_bchunk;
    L.lr_R = d_lr_R, L.lr_P = d_lr_P, L.lr_base = d_lr_base;
    L.pb0 = d_pb0, L.cb_n = d_cb_n, L.db0 = d_db0, L.rb_n = d_rb_n;
    L.ia_desc = d_ia_desc, L.tb_desc = d_tb_desc, L.tb_rows = d_tb_rows;
    L.ev_blk0 = d_ev0, L.ev_inst = d_ev_inst;
    L.a_nchunks = a_nchunks, L.t_nchunks = t_nchunks, L.ab_blocks = ia_blocks, L.tb_blocks = tb_blocks;
    L.ev_blocks = ev_blocks;
    P.a_rp = a_rp, P.a_ci = a_ci, P.a_chunk_row = ia_chunk_row, P.a_chunk_cls = ia_chunk_cls, P.a_val = a_v;
    P.t_rp = t_rp, P.t_ci = t_ci, P.t_chunk_row = t_chunk_row, P.t_chunk_cls = t_chunk_cls, P.t_val = t_v;
    P.c = cT, P.l = lT, P.u = uT, P.b = bT, P.sense = sense, P.Dr = Dr, P.Dc = Dc;
    for (int q = 0; q < 2; ++q) P.x[q] = xs[q], P.y[q] = ys[q], P.ax[q] = axs[q];
    P.aty = aty, P.xbar = xbar, P.ybar = ybar, P.axbar = axbar, P.atybar = atybar, P.xa = xa, P.ya = ya;
    P.p_dual = p_dual, P.p_primal = p_primal, P.p_restart = p_restart, P.p_eval = p_eval, P.part = part;
    P.st = st, P.ndone = ndone;
  }

  // ---------------------------------------------------------------------------------------------
  // SpMV schedule
  // ---------------------------------------------------------------------------------------------
  void make_chunks(int cap) {
    std::vector<int32_t> ra, rt;
    std::vector<int8_t> ca, ct;
    h_a_chunk0.assign(1, 0), h_t_chunk0.assign(1, 0);
    for (int q = 0; q < K; ++q) {
      if (ra.empty()) ra.push_back(h_row0[q]);
      build_chunks(h_arp.data(), h_row0[q], h_row0[q + 1], cap, ra, ca);
      h_a_chunk0.push_back((int32_t)ca.size());
      if (rt.empty()) rt.push_back(h_col0[q]);
      build_chunks(h_trp.data(), h_col0[q], h_col0[q + 1], cap, rt, ct);
      h_t_chunk0.push_back((int32_t)ct.size());
    }
    for (void *p : {(void *)a_chunk_row, (void *)t_chunk_row, (void *)a_chunk_cls, (void *)t_chunk_cls,
                    (void *)d_a_chunk0, (void *)d_t_chunk0, (void *)d_ab0, (void *)d_ab_inst, (void *)d_tb0,
                    (void *)d_tb_inst, (void *)d_a_bchunk, (void *)d_t_bchunk, (void *)ia_chunk_row,
                    (void *)ia_chunk_cls, (void *)d_ia_ab0, (void *)d_ia_ab_inst, (void *)d_ia_bchunk})
      if (p) mem.release(p);
    a_chunk_row = alloc_upload(ra), t_chunk_row = alloc_upload(rt);
    a_chunk_cls = alloc_upload(ca), t_chunk_cls = alloc_upload(ct);
    d_a_chunk0 = alloc_upload(h_a_chunk0), d_t_chunk0 = alloc_upload(h_t_chunk0);
    a_nchunks = (int)ca.size(), t_nchunks = (int)ct.size();
    chunk_nnz = cap;
    // Work blocks: an instance of weight w (nonzeros + rows: every row has an epilogue) gets
    // ceil(w / kMinBlockWeight) blocks per side, at most work_blocks, at least one and at most one
    // per chunk. The count depends on the instance alone, so an instance solved in a batch groups
    // its FP64 partial sums exactly as it does solved alone (same chunk size), and follows the same
    // trajectory bit for bit. Inside an instance each block takes a contiguous run of chunks of about
    // equal weight; a chunk heavier than a block's share (one very long row) gets a block of its own.
    std::vector<int32_t> ab_inst, tb_inst, a_bchunk, t_bchunk;
    auto blocks_for = [&](const std::vector<int32_t> &rp, const std::vector<int32_t> &crow,
                          const std::vector<int32_t> &ch0, std::vector<int32_t> &b0, std::vector<int32_t> &binst,
                          std::vector<int32_t> &bchunk) {
      const int nch = ch0.back();
      std::vector<int64_t> wpre((size_t)nch + 1, 0);  // prefix of chunk weights (global)
      for (int c = 0; c < nch; ++c)
        wpre[c + 1] = wpre[c] + (rp[crow[c + 1]] - rp[crow[c]]) + (crow[c + 1] - crow[c]);
      b0.assign(1, 0);
      binst.clear();
      bchunk.clear();
      for (int q = 0; q < K; ++q) {
        const int c0 = ch0[q], c1 = ch0[q + 1];
        const int64_t wq = wpre[c1] - wpre[c0];
        int64_t nbq = std::min<int64_t>(work_blocks, (wq + kMinBlockWeight - 1) / kMinBlockWeight);
        nbq = std::max<int64_t>(1, std::min<int64_t>(nbq, std::max(c1 - c0, 1)));
        int c = c0;
        for (int64_t lb = 0; lb < nbq; ++lb) {
          // first chunk whose start lies at or past this block's share of the weight
          const int64_t target = wpre[c0] + (wq * lb + nbq - 1) / nbq;
          while (c < c1 && wpre[c] < target) ++c;
          bchunk.push_back(c);
          binst.push_back(q);
        }
        b0.push_back(b0.back() + (int32_t)nbq);
      }
      bchunk.push_back(nch);
    };
    blocks_for(h_arp, ra, h_a_chunk0, h_ab0, ab_inst, a_bchunk);
    blocks_for(h_trp, rt, h_t_chunk0, h_tb0, tb_inst, t_bchunk);
    ab_blocks = h_ab0.back(), tb_blocks = h_tb0.back();
    d_ab0 = alloc_upload(h_ab0), d_ab_inst = alloc_upload(ab_inst);
    d_tb0 = alloc_upload(h_tb0), d_tb_inst = alloc_upload(tb_inst);
    d_a_bchunk = alloc_upload(a_bchunk), d_t_bchunk = alloc_upload(t_bchunk);
    h_t_bchunk = t_bchunk;

    // Iteration layout of the A side (k_dual). Per instance: a chunk over its long rows that no
    // block takes (their sums come from the column panels), the chunks of its other rows shared out
    // by weight exactly as above, and one block per kBlock long rows. Blocks are given as (first,
    // end) chunk pairs, long-row block j as (-1 - j, -1 - j). Without long rows this is the layout
    // above, block for block.
    std::vector<int32_t> ri, ia_inst, ia_bc, cstart((size_t)K), cend((size_t)K);
    std::vector<int8_t> ci8;
    for (int q = 0; q < K; ++q) {
      const int32_t rs = h_row0[q] + h_lr_R[q];
      if (ri.empty()) ri.push_back(h_row0[q]);
      if (h_lr_R[q] > 0) ri.push_back(rs), ci8.push_back(6);
      cstart[q] = (int32_t)ci8.size();
      build_chunks(h_arp.data(), rs, h_row0[q + 1], cap, ri, ci8);
      cend[q] = (int32_t)ci8.size();
    }
    {
      const int nch = (int)ci8.size();
      std::vector<int64_t> wpre((size_t)nch + 1, 0);
      for (int c = 0; c < nch; ++c)
        wpre[c + 1] = wpre[c] + (h_arp[ri[c + 1]] - h_arp[ri[c]]) + (ri[c + 1] - ri[c]);
      h_ia_ab0.assign(1, 0);
      for (int q = 0; q < K; ++q) {
        const int c0 = cstart[q], c1 = cend[q];
        const int64_t wq = wpre[c1] - wpre[c0];
        int64_t nbq = std::min<int64_t>(work_blocks, (wq + kMinBlockWeight - 1) / kMinBlockWeight);
        nbq = std::max<int64_t>(1, std::min<int64_t>(nbq, std::max(c1 - c0, 1)));
        std::vector<int32_t> starts;
        int c = c0;
        for (int64_t lb = 0; lb < nbq; ++lb) {
          const int64_t target = wpre[c0] + (wq * lb + nbq - 1) / nbq;
          while (c < c1 && wpre[c] < target) ++c;
          starts.push_back(c);
        }
        // long-row blocks spread evenly among the chunk blocks: consecutive blocks of an instance
        // run on the same XCD (xcd_remap), so a run of long-row blocks at the end would load one XCD
        const int nlong = (h_lr_R[q] + kBlock - 1) / kBlock;
        const int64_t nb = nbq + nlong;
        int64_t lb = 0, j = 0;
        for (int64_t b = 0; b < nb; ++b) {
          if (j < ((b + 1) * nlong) / nb) {
            ia_bc.push_back((int32_t)(-1 - j)), ia_bc.push_back((int32_t)(-1 - j)), ++j;
          } else {
            ia_bc.push_back(starts[lb]), ia_bc.push_back(lb + 1 < nbq ? starts[lb + 1] : c1), ++lb;
          }
          ia_inst.push_back(q);
        }
        h_ia_ab0.push_back(h_ia_ab0.back() + (int32_t)nb);
      }
    }
    ia_blocks = h_ia_ab0.back();
    h_ia_bc = ia_bc;
    ia_chunk_row = alloc_upload(ri), ia_chunk_cls = alloc_upload(ci8);
    d_ia_ab0 = alloc_upload(h_ia_ab0), d_ia_ab_inst = alloc_upload(ia_inst);
    d_ia_bchunk = alloc_upload(ia_bc);
  }

  template <typename V, typename X, typename Acc, typename Y>
  void spmv_chunks(int trans, const X *x, Y *y) {
    const int32_t *rp = trans ? t_rp : a_rp;
    const int32_t *ci = trans ? t_ci : a_ci;
    const V *v;
    if constexpr (sizeof(V) == sizeof(double)) v = (const V *)(trans ? t_v64 : a_v64);
    else v = (const V *)(trans ? t_v : a_v);
    const int nch = trans ? t_nchunks : a_nchunks;
    if (nch <= 0) return;
    hipLaunchKernelGGL((k_spmv<V, X, Acc, Y>), dim3(trans ? tb_blocks : ab_blocks), dim3(kBlock), 0, stream, rp, ci,
                       v, (const int32_t *)(trans ? t_chunk_row : a_chunk_row),
                       (const int8_t *)(trans ? t_chunk_cls : a_chunk_cls), (const int32_t *)(trans ? d_tb0 : d_ab0),
                       (const int32_t *)(trans ? d_tb_inst : d_ab_inst),
                       (const int32_t *)(trans ? d_t_bchunk : d_a_bchunk), x, y);
  }
  void spmv_T(int trans, const T *x, T *y) { spmv_chunks<T, T, double, T>(trans, x, y); }

  // Autotuner: time A x and A'y for each candidate chunk size; keep the smallest size unless
  // another is at least 15 % faster. The choice is cached per sparsity signature.
  void choose_schedule() {
    if (opt.tile_nnz > 0) {
      bool ok = false;
      for (int c : kChunkCandidates) ok |= (c == opt.tile_nnz);
      if (!ok) raise(PDLP_ERR_ARG, "tile_nnz must be one of 512, 1024, 2048, 4096 (or 0 = autotune)");
      make_chunks(opt.tile_nnz);
      return;
    }
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune_cache.find(sig);
      if (it != g_tune_cache.end()) {
        make_chunks(it->second);
        return;
      }
    }
    int pick = kChunkCandidates[0];
    if (nnz >= 200000) {
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      float best = 1e30f;
      std::vector<std::pair<int, float>> times;
      for (int cand : kChunkCandidates) {
        make_chunks(cand);
        spmv_T(0, xs[0], axs[0]);
        spmv_T(1, ys[0], aty);
        HIPCHK(hipEventRecord(e0, stream));
        for (int r = 0; r < 5; ++r) {
          spmv_T(0, xs[0], axs[0]);
          spmv_T(1, ys[0], aty);
        }
        HIPCHK(hipEventRecord(e1, stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        times.push_back({cand, ms});
        best = std::min(best, ms);
      }
      // Keep the finest size unless another is clearly faster: the choice must not flip between
      // runs on timing noise, because the block partition (and with it the grouping of the FP64
      // partial sums, hence the rounding of the whole trajectory) follows from it.
      pick = times[0].first;
      for (auto &t : times)
        if (t.second <= best * 1.0001f && t.second < 0.85f * times[0].second) pick = t.first;
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    make_chunks(pick);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[sig] = pick;
  }

  // ---------------------------------------------------------------------------------------------
  // Iteration launches
  // ---------------------------------------------------------------------------------------------
  void launch_panels() {
    if (PQ.nwg > 0) hipLaunchKernelGGL(k_panel<T>, dim3(PQ.nwg), dim3(kPanelBlock), 0, stream, P, PQ);
  }
  void launch_primal() {
    if (chunk_primal) hipLaunchKernelGGL(k_primal<T>, dim3(tb_blocks), dim3(kBlock), 0, stream, P);
    if constexpr (sizeof(T) == sizeof(float)) {
      if (CQ.nwg > 0) hipLaunchKernelGGL(k_primal_cb<T>, dim3(CQ.nwg), dim3(kCbBlock), 0, stream, P, CQ);
    }
  }
  void launch_dual() {
    if (chunk_dual) hipLaunchKernelGGL(k_dual<T>, dim3(ia_blocks), dim3(kBlock), 0, stream, P);
    if constexpr (sizeof(T) == sizeof(float)) {
      if (RQ.nwg > 0) hipLaunchKernelGGL(k_dual_rb<T>, dim3(RQ.nwg), dim3(kCbBlock), 0, stream, P, RQ);
    }
  }
  void launch_attempt() {
    launch_panels();
    launch_dual();
    launch_step();
    launch_primal();
  }
  void launch_step() {
    hipLaunchKernelGGL(k_step, dim3(K), dim3(kStepBlock), 0, stream, P.L, (const double *)p_dual,
                       (const double *)p_primal, (const double *)p_restart, st, ndone);
  }
  void launch_eval(int mode) {
    hipLaunchKernelGGL(k_eval<T>, dim3(ev_blocks), dim3(kBlock), 0, stream, P);
    hipLaunchKernelGGL(k_eval_fin, dim3(K), dim3(kBlock), 0, stream, P.L, (const double *)p_eval, st, ndone, mode);
  }
  void launch_restart() { hipLaunchKernelGGL(k_restart<T>, dim3(ev_blocks), dim3(kBlock), 0, stream, P); }
  // Evaluation and restart at the end of an interval, with the snapshot kernels around the restart
  // when snapshots are on.
  void launch_eval_restart() {
    launch_eval(kEvalChunk);
    if (snap.K > 0)
      hipLaunchKernelGGL(k_snap_pick, dim3(grid_for(K)), dim3(kBlock), 0, stream, K, (const State *)st, snap);
    launch_restart();
    if (snap.K > 0) hipLaunchKernelGGL(k_snap_copy<T>, dim3(ev_blocks), dim3(kBlock), 0, stream, P, snap);
  }
  // Before each evaluation: the average update an accepted attempt may have left pending (paired
  // updates), then, in FP32, the products of the averages. Kept up to date by the same weighted
  // updates as the averages themselves, they would drift from A x-bar and A'y-bar by accumulated
  // rounding; recomputed, the average's KKT error and the caches a restart to the average hands on
  // are those of the averaged point itself. (FP64 keeps the updates.)
  void refresh_averages() {
    if constexpr (sizeof(T) == sizeof(float)) {
      hipLaunchKernelGGL(k_avg_flush<T>, dim3(ev_blocks), dim3(kBlock), 0, stream, P);
      spmv_chunks<T, double, double, T>(0, xbar, axbar);
      spmv_chunks<T, double, double, T>(1, ybar, atybar);
    }
  }
  void launch_chunk_body() {
    for (int r = 0; r < opt.eval_every; ++r) launch_attempt();
    refresh_averages();
    launch_eval_restart();
  }
  // Direct launches whose dispatch packets record events (pool `slot`): per attempt the start and
  // stop of k_panel, of k_dual and of the primal kernels (k_primal and / or k_primal_cb: the first
  // one's start, the last one's stop). The timestamps are taken by the kernels' own dispatches, so
  // the durations are the kernels', without separate marker packets.
  void launch_chunk_timed(int slot) {
    auto &pool = tev[slot];
    if (pool.empty()) {
      pool.resize((size_t)opt.eval_every * 6);
      for (auto &e : pool) HIPCHK(hipEventCreate(&e));
    }
    for (int r = 0; r < opt.eval_every; ++r) {
      hipEvent_t *e = &pool[(size_t)r * 6];
      if (PQ.nwg > 0) hipExtLaunchKernelGGL(k_panel<T>, dim3(PQ.nwg), dim3(kPanelBlock), 0, stream, e[0], e[1], 0, P, PQ);
      const bool rb = sizeof(T) == sizeof(float) && RQ.nwg > 0;
      if (chunk_dual)
        hipExtLaunchKernelGGL(k_dual<T>, dim3(ia_blocks), dim3(kBlock), 0, stream, e[2], rb ? nullptr : e[3], 0, P);
      if constexpr (sizeof(T) == sizeof(float)) {
        if (rb)
          hipExtLaunchKernelGGL(k_dual_rb<T>, dim3(RQ.nwg), dim3(kCbBlock), 0, stream, chunk_dual ? nullptr : e[2],
                                e[3], 0, P, RQ);
      }
      launch_step();
      const bool cb = sizeof(T) == sizeof(float) && CQ.nwg > 0;
      if (chunk_primal)
        hipExtLaunchKernelGGL(k_primal<T>, dim3(tb_blocks), dim3(kBlock), 0, stream, e[4], cb ? nullptr : e[5], 0, P);
      if constexpr (sizeof(T) == sizeof(float)) {
        if (cb)
          hipExtLaunchKernelGGL(k_primal_cb<T>, dim3(CQ.nwg), dim3(kCbBlock), 0, stream,
                                chunk_primal ? nullptr : e[4], e[5], 0, P, CQ);
      }
      HIPCHK(hipGetLastError());
    }
    refresh_averages();
    launch_eval_restart();
    HIPCHK(hipGetLastError());
  }
  // Add the durations recorded in pool `slot` (its chunk has completed): kernel 0 = the dual
  // kernels (k_dual and / or k_dual_rb), 1 = the primal kernels (k_primal and / or k_primal_cb),
  // 2 = k_panel (counted only when the handle uses column panels), 3 = the primal kernels again when
  // they include k_primal_cb (counted only when the handle uses column blocks), 4 = the dual kernels
  // again when they include k_dual_rb (counted only when the handle uses row blocks).
  void collect_times(int slot) {
    auto &pool = tev[slot];
    static const int kFrom[5] = {2, 4, 0, 4, 2}, kTo[5] = {3, 5, 1, 5, 3};
    for (int r = 0; r < opt.eval_every && !pool.empty(); ++r)
      for (int k = 0; k < 5; ++k) {
        if ((k == 2 && PQ.nwg == 0) || (k == 3 && CQ.nwg == 0) || (k == 4 && RQ.nwg == 0)) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, pool[(size_t)r * 6 + kFrom[k]], pool[(size_t)r * 6 + kTo[k]]));
        t_ms[k] += ms;
        t_launches[k] += 1;
      }
  }

  void run_chunk(int64_t ch) {
    if (opt.kernel_timing) {
      launch_chunk_timed((int)(ch & 1));
      return;
    }
    if (!opt.use_graphs) {
      launch_chunk_body();
      HIPCHK(hipGetLastError());
      return;
    }
    if (!graph) {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      launch_chunk_body();
      HIPCHK(hipStreamEndCapture(stream, &g));
      HIPCHK(hipGraphInstantiate(&graph, g, nullptr, nullptr, 0));
      HIPCHK(hipGraphDestroy(g));
    }
    HIPCHK(hipGraphLaunch(graph, stream));
  }

  // ---------------------------------------------------------------------------------------------
  // Solve
  // ---------------------------------------------------------------------------------------------
  // Stage warm starts (original space; NULL entries = cold) and write the start point.
  bool stage_start(const double *const *x0s, const double *const *y0s) {
    bool any = false;
    for (int q = 0; q < K; ++q) any |= (x0s && x0s[q]) || (y0s && y0s[q]);
    if (!any) {
      start_point(nullptr, nullptr, xs[0], ys[0]);
      return false;
    }
    const hipMemcpyKind kind = opt.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(hipMemsetAsync(stage_n, 0, sizeof(double) * (size_t)std::max(n, 1), stream));
    HIPCHK(hipMemsetAsync(stage_m, 0, sizeof(double) * (size_t)std::max(m, 1), stream));
    for (int q = 0; q < K; ++q) {
      const int32_t nq = h_col0[q + 1] - h_col0[q], mq = h_row0[q + 1] - h_row0[q];
      if (x0s && x0s[q] && nq)
        HIPCHK(hipMemcpyAsync(stage_n + h_col0[q], x0s[q], sizeof(double) * (size_t)nq, kind, stream));
      if (y0s && y0s[q] && mq)
        HIPCHK(hipMemcpyAsync(stage_m + h_row0[q], y0s[q], sizeof(double) * (size_t)mq, kind, stream));
    }
    gather64(n, stage_n, d_perm_c, xd);  // external -> internal numbering
    gather64(m, stage_m, d_perm_r, yd);
    start_point(xd, yd, xs[0], ys[0]);
    return true;
  }
  template <typename U>
  void start_point(const double *dx, const double *dy, U *x, U *y) {
    hipLaunchKernelGGL(k_init_point<U>, dim3(grid_for(std::max(m, n))), dim3(kBlock), 0, stream, m, n, dx, dy,
                       (const double *)Dr, (const double *)Dc, (const double *)l64, (const double *)u64,
                       (const uint8_t *)sense, x, y);
    HIPCHK(hipGetLastError());
  }

  void gather64(int len, const double *src, const int32_t *idx, double *dst) {
    if (len <= 0) return;
    hipLaunchKernelGGL(k_gather64, dim3(grid_for(len)), dim3(kBlock), 0, stream, len, src, idx, dst);
  }

  void upload_state() { upload(st, h_st.data(), K); }
  void read_state() {
    download(h_st.data(), st, K);
    sync();
  }
  int32_t count_done() {
    int32_t c = 0;
    for (auto &s : h_st) c += s.done;
    return c;
  }

  void solve(double tol, int64_t iter_limit, const double *const *x0s, const double *const *y0s,
             const double *omega0s) {
    const auto t0 = std::chrono::steady_clock::now();
    iter_limit = std::max<int64_t>(iter_limit, 1);
    for (int q = 0; q < K; ++q) {
      State &s = h_st[q];
      std::memset(&s, 0, sizeof(State));
      s.eta = eta0[q];
      s.omega = (omega0s && omega0s[q] > 0.0) ? omega0s[q] : omega_default[q];
      s.tol = tol > 0.0 ? tol : -1.0;
      s.nb = nb[q], s.nc = nc[q];
      s.kkt_prev = INFINITY;
      s.iter_limit = iter_limit;
      s.eval_every = opt.eval_every;
      s.restart_mode = kToCurrent;
      // FP32 pairs the average updates of consecutive accepted attempts (FP64 also updates the
      // averages' products in k_primal and keeps one update per attempt)
      s.pair_avg = (sizeof(T) == sizeof(float) && !opt.single_avg_updates) ? 1 : 0;
    }
    upload_state();
    HIPCHK(hipMemsetAsync(ndone, 0, sizeof(int32_t), stream));
    if (snap.K > 0) HIPCHK(hipMemsetAsync(snap.taken, 0, sizeof(int32_t) * (size_t)K, stream));
    for (int k = 0; k < 5; ++k) t_launches[k] = 0, t_ms[k] = 0.0;
    const bool warm = stage_start(x0s, y0s);
    std::vector<int> fallback((size_t)K, 0), warm_q((size_t)K, 0);
    for (int q = 0; q < K; ++q) warm_q[q] = (x0s && x0s[q]) || (y0s && y0s[q]);
    spmv_T(0, xs[0], axs[0]);
    spmv_T(1, ys[0], aty);
    if (warm && opt.warm_fallback) {
      // cold start in the average slots; compare the relative KKT errors of both points
      start_point(nullptr, nullptr, xbar, ybar);
      spmv_chunks<T, double, double, T>(0, xbar, axbar);
      spmv_chunks<T, double, double, T>(1, ybar, atybar);
      launch_eval(kEvalPoint);
      HIPCHK(hipGetLastError());
      read_state();
      bool any = false;
      for (int q = 0; q < K; ++q)
        if (warm_q[q] && !(h_st[q].cand_rel[0] < h_st[q].cand_rel[1])) {
          fallback[q] = 1, any = true;
          const int32_t nq = h_col0[q + 1] - h_col0[q], mq = h_row0[q + 1] - h_row0[q];
          if (nq) HIPCHK(hipMemsetAsync(stage_n + h_col0[q], 0, sizeof(double) * (size_t)nq, stream));
          if (mq) HIPCHK(hipMemsetAsync(stage_m + h_row0[q], 0, sizeof(double) * (size_t)mq, stream));
          // 1: the cold start in full; 2: the cold point with the given primal weight kept
          if (omega0s && omega0s[q] > 0.0 && opt.warm_fallback != 2) h_st[q].omega = omega_default[q];
        }
      if (any) {
        gather64(n, stage_n, d_perm_c, xd);
        gather64(m, stage_m, d_perm_r, yd);
        start_point(xd, yd, xs[0], ys[0]);
        spmv_T(0, xs[0], axs[0]);
        spmv_T(1, ys[0], aty);
        upload_state();
      }
    }
    launch_eval(kEvalInit);
    launch_restart();
    HIPCHK(hipGetLastError());

    std::vector<int> checks((size_t)K, 0);
    std::vector<double> tol_int((size_t)K, tol);
    while (true) {
      run_loop(iter_limit);
      read_state();
      finalize();
      read_state();
      bool resume = false;
      for (int q = 0; q < K; ++q) {
        State &s = h_st[q];
        if (s.done != 1) continue;
        const double rk = std::max(s.rel_p, std::max(s.rel_d, s.rel_gap));
        if (checks[q] == 0 || s.status == PDLP_STATUS_OPTIMAL) checks[q] += (s.status != 0);
        if (s.status == PDLP_STATUS_OPTIMAL && tol > 0.0 && !(rk <= tol)) {
          if (checks[q] <= kMaxResumes && s.k < iter_limit) {
            // the FP64 recomputation from the FP64 matrix disagrees with the in-loop evaluation:
            // continue this instance from the same state with the internal tolerance tightened by
            // the observed miss (at least 20 %), so a point that just missed costs a short resume
            tol_int[q] *= std::min(0.8, 0.95 * tol / rk);
            s.done = 0, s.status = 0, s.stop = 0, s.tol = tol_int[q];
            resume = true;
          } else {
            s.status = PDLP_STATUS_ITER_LIMIT;
          }
        }
      }
      if (!resume) break;
      int32_t nd = count_done();
      upload_state();
      upload(ndone, &nd, 1);
    }
    const auto t1 = std::chrono::steady_clock::now();
    const double secs = std::chrono::duration<double>(t1 - t0).count();
    for (int q = 0; q < K; ++q) {
      const State &s = h_st[q];
      pdlp_result &r = last[q];
      r = pdlp_result{};
      r.status = s.status;
      r.restarts = s.restarts;
      r.iterations = s.k;
      r.rel_primal = s.rel_p;
      r.rel_dual = s.rel_d;
      r.rel_gap = s.rel_gap;
      r.primal_obj = s.pobj;
      r.dual_obj = s.dobj;
      r.omega = s.omega;
      r.eta = s.eta;
      r.solve_seconds = secs;
      r.used_average = s.which;
      r.warm_started = warm_q[q] && !fallback[q];
      r.fallback_used = fallback[q];
      r.final_checks = checks[q];
    }
    solved = true;
    if (opt.verbose)
      for (int q = 0; q < std::min(K, 8); ++q)
        fprintf(stderr, "[pdlp] inst %d status %d iters %lld restarts %d rel_p %.3e rel_d %.3e gap %.3e obj %.10g (%.3f s)\n",
                q, last[q].status, (long long)last[q].iterations, last[q].restarts, last[q].rel_primal,
                last[q].rel_dual, last[q].rel_gap, last[q].primal_obj, secs);
  }

  // Launch evaluation intervals until every instance is done. Two intervals are kept in flight:
  // the host waits for the done counter of interval c-1 while interval c runs; an interval launched
  // after all instances finished does no work.
  void run_loop(int64_t iter_limit) {
    const int64_t max_chunks = iter_limit / opt.eval_every + 3;
    int64_t ch = 0;
    // verbose >= 2 (or PDLP_TRACE_EVALS=<period>: every <period> evaluations): print the relative
    // errors of both candidates of the first instances after each evaluation (one interval in flight
    // then; the results do not change)
    static const char *trace_env = getenv("PDLP_TRACE_EVALS");
    const int64_t trace_every = opt.verbose >= 2 ? 1 : trace_env ? std::max<int64_t>(1, atoll(trace_env)) : 0;
    for (; ch < max_chunks; ++ch) {
      run_chunk(ch);
      if (trace_every && ch % trace_every == 0) {
        read_state();
        for (int q = 0; q < std::min(K, 4); ++q) {
          const State &s = h_st[q];
          fprintf(stderr, "[pdlp-trace] inst %d k %lld restarts %d omega %.4e eta %.4e | cur p %.3e d %.3e g %.3e | avg p %.3e d %.3e g %.3e%s\n",
                  q, (long long)s.k, s.restarts, s.omega, s.eta, s.ev_rel[0], s.ev_rel[1], s.ev_rel[2], s.ev_rel[3],
                  s.ev_rel[4], s.ev_rel[5], s.done ? " done" : "");
        }
      }
      HIPCHK(hipMemcpyAsync(&h_flags[ch & 1], ndone, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
      HIPCHK(hipEventRecord(ev[ch & 1], stream));
      if (ch >= 1) {
        HIPCHK(hipEventSynchronize(ev[(ch - 1) & 1]));
        if (opt.kernel_timing) collect_times((int)((ch - 1) & 1));
        if (h_flags[(ch - 1) & 1] >= K) break;  // chunk ch found every instance done: not timed
      }
    }
    sync();
    if (opt.kernel_timing && ch == max_chunks) collect_times((int)((ch - 1) & 1));
  }

  void finalize() {
    hipLaunchKernelGGL(k_unscale<T>, dim3(ev_blocks), dim3(kBlock), 0, stream, P, xd, yd, x_out, y_out);
    spmv_chunks<double, double, double, double>(0, xd, ax64);
    spmv_chunks<double, double, double, double>(1, yd, aty64);
    Final64 F{xd, yd, ax64, aty64, c64, b64, l64, u64, rc_out, p_final};
    hipLaunchKernelGGL(k_final_residuals<T>, dim3(ev_blocks), dim3(kBlock), 0, stream, P, F);
    hipLaunchKernelGGL(k_final_fin, dim3(K), dim3(kBlock), 0, stream, P.L, (const double *)p_final, st);
    gather64(n, x_out, d_inv_c, x_ext);  // internal -> external numbering
    gather64(m, y_out, d_inv_r, y_ext);
    gather64(n, rc_out, d_inv_c, rc_ext);
    HIPCHK(hipGetLastError());
  }

  void get(int q, double *x, double *y, double *rc, pdlp_result *res) {
    if (!solved) raise(PDLP_ERR_STATE, "get before solve");
    if (q < 0 || q >= K) raise(PDLP_ERR_ARG, "instance index out of range");
    const hipMemcpyKind kind = opt.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const int32_t c0 = h_col0[q], nq = h_col0[q + 1] - c0, r0 = h_row0[q], mq = h_row0[q + 1] - r0;
    if (x && nq) HIPCHK(hipMemcpyAsync(x, x_ext + c0, sizeof(double) * (size_t)nq, kind, stream));
    if (y && mq) HIPCHK(hipMemcpyAsync(y, y_ext + r0, sizeof(double) * (size_t)mq, kind, stream));
    if (rc && nq) HIPCHK(hipMemcpyAsync(rc, rc_ext + c0, sizeof(double) * (size_t)nq, kind, stream));
    sync();
    if (res) *res = last[q];
  }

  // Reference snapshots: k slots per instance (k = 0: off) for the restart points of later solves
  // whose relative KKT error is at most rel_tol. Replaces the ring (and what it held); the interval
  // graph is captured again with or without the snapshot kernels.
  void set_snapshots(int32_t k, double rel_tol) {
    if (k < 0 || std::isnan(rel_tol)) raise(PDLP_ERR_ARG, "snapshots: k must be >= 0 and rel_tol not NaN");
    sync();
    for (void *q : {(void *)snap.x, (void *)snap.y, (void *)snap.attempt, (void *)snap.rel, (void *)snap.taken,
                    (void *)snap.slot})
      if (q) mem.release(q);
    snap = Snap{};
    if (graph) {
      HIPCHK(hipGraphExecDestroy(graph));
      graph = nullptr;
    }
    if (k == 0) return;
    snap.x = mem.alloc<double>((int64_t)k * n);
    snap.y = mem.alloc<double>((int64_t)k * m);
    snap.attempt = mem.alloc<int64_t>((int64_t)K * k);
    snap.rel = mem.alloc<double>((int64_t)K * k);
    snap.taken = mem.alloc<int32_t>(K);
    snap.slot = mem.alloc<int32_t>(K);
    HIPCHK(hipMemsetAsync(snap.taken, 0, sizeof(int32_t) * (size_t)K, stream));
    sync();
    snap.K = k, snap.n = n, snap.m = m, snap.rel_tol = rel_tol;
  }

  // Snapshots of instance q held after the last solve, oldest first, in the caller's numbering: at
  // most `cap` of them (the newest); *count = the number written.
  void get_snapshots(int q, int32_t cap, double *x, double *y, int64_t *attempt, double *rel, int32_t *count) {
    if (!solved) raise(PDLP_ERR_STATE, "snapshots before solve");
    if (q < 0 || q >= K) raise(PDLP_ERR_ARG, "instance index out of range");
    if (cap < 0 || !count) raise(PDLP_ERR_ARG, "snapshots: cap must be >= 0 and count not NULL");
    *count = 0;
    if (snap.K == 0 || cap == 0) return;
    int32_t taken = 0;
    std::vector<int64_t> h_att((size_t)snap.K);
    std::vector<double> h_rel((size_t)snap.K);
    download(&taken, snap.taken + q, 1);
    download(h_att.data(), snap.attempt + (size_t)q * snap.K, snap.K);
    download(h_rel.data(), snap.rel + (size_t)q * snap.K, snap.K);
    sync();
    const int32_t held = std::min(taken, snap.K), out = std::min(held, cap);
    const hipMemcpyKind kind = opt.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const int32_t c0 = h_col0[q], nq = h_col0[q + 1] - c0, r0 = h_row0[q], mq = h_row0[q + 1] - r0;
    for (int32_t i = 0; i < out; ++i) {
      const int32_t s = (taken - out + i) % snap.K;  // oldest of the newest `out` first
      if (attempt) attempt[i] = h_att[(size_t)s];
      if (rel) rel[i] = h_rel[(size_t)s];
      if (x && nq) {
        gather64(n, snap.x + (size_t)s * n, d_inv_c, stage_n);  // internal -> external numbering
        HIPCHK(hipMemcpyAsync(x + (size_t)i * nq, stage_n + c0, sizeof(double) * (size_t)nq, kind, stream));
      }
      if (y && mq) {
        gather64(m, snap.y + (size_t)s * m, d_inv_r, stage_m);
        HIPCHK(hipMemcpyAsync(y + (size_t)i * mq, stage_m + r0, sizeof(double) * (size_t)mq, kind, stream));
      }
    }
    HIPCHK(hipGetLastError());
    sync();
    *count = out;
  }

  // Original-space product y = A x = Dr^-1 A~ Dc^-1 x (trans = 0) or y = A'x (trans = 1), in the
  // caller's numbering.
  // A x as the iteration forms it: long rows by column panels (k_panel_x, k_long_sum), the other
  // rows by the chunks of the iteration layout.
  void spmv_iter(const T *x, T *y) {
    if (PQ.nwg > 0) {
      hipLaunchKernelGGL(k_panel_x<T>, dim3(PQ.nwg), dim3(kPanelBlock), 0, stream, P.L, PQ, x, part);
      hipLaunchKernelGGL(k_long_sum<T>, dim3(ia_blocks), dim3(kBlock), 0, stream, P.L, (const double *)part, y);
    }
    hipLaunchKernelGGL((k_spmv_pairs<T, T, double, T>), dim3(ia_blocks), dim3(kBlock), 0, stream, (const int32_t *)a_rp,
                       (const int32_t *)a_ci, (const T *)a_v, (const int32_t *)ia_chunk_row, (const int8_t *)ia_chunk_cls,
                       (const int32_t *)d_ia_ab0, (const int32_t *)d_ia_ab_inst, (const int32_t *)d_ia_bchunk, x, y);
    if constexpr (sizeof(T) == sizeof(float)) {  // the row-block instances, over the chunk engine's result
      if (RQ.nwg > 0) hipLaunchKernelGGL(k_rb_x<T>, dim3(RQ.nwg), dim3(kCbBlock), 0, stream, P.L, RQ, x, y);
    }
  }

  // A'y as the iteration forms it: the column-block instances by k_cb_x over the chunk engine's
  // result for all instances.
  void spmv_iter_t(const T *yv, T *out) {
    spmv_T(1, yv, out);
    if constexpr (sizeof(T) == sizeof(float)) {
      if (CQ.nwg > 0) hipLaunchKernelGGL(k_cb_x<T>, dim3(CQ.nwg), dim3(kCbBlock), 0, stream, P.L, CQ, yv, out);
    }
  }

  void spmv(int trans_mode, const double *x, double *y) {
    const int trans = trans_mode == 1 || trans_mode == 3;
    const int in = trans ? m : n, out = trans ? n : m;
    double *sin = trans ? stage_m : stage_n;
    double *xin = trans ? yd : xd;
    double *yint = trans ? aty64 : ax64;
    double *sout = trans ? stage_n : stage_m;
    T *tin = trans ? tmp_m : tmp_n;
    T *tout = trans ? tmp_n : tmp_m;
    const hipMemcpyKind k_in = opt.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind k_out = opt.device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (in) HIPCHK(hipMemcpyAsync(sin, x, sizeof(double) * (size_t)in, k_in, stream));
    gather64(in, sin, trans ? d_perm_r : d_perm_c, xin);
    hipLaunchKernelGGL(k_div_to<T>, dim3(grid_for(in)), dim3(kBlock), 0, stream, in, (const double *)xin,
                       (const double *)(trans ? Dr : Dc), tin);
    if (trans_mode == 2) spmv_iter(tin, tout);
    else if (trans_mode == 3) spmv_iter_t(tin, tout);
    else spmv_T(trans, tin, tout);
    hipLaunchKernelGGL(k_div_from<T>, dim3(grid_for(out)), dim3(kBlock), 0, stream, out, (const T *)tout,
                       (const double *)(trans ? Dc : Dr), yint);
    gather64(out, yint, trans ? d_inv_c : d_inv_r, sout);
    HIPCHK(hipGetLastError());
    if (out) HIPCHK(hipMemcpyAsync(y, sout, sizeof(double) * (size_t)out, k_out, stream));
    sync();
  }

  // New bounds for instance q (caller's numbering): validated like create's, scaled and renumbered
  // into the iteration copies exactly as create does, so a later solve behaves as on a new handle
  // made with these bounds. Matrix, costs, scaling and schedule are kept.
  void update_bounds(int q, const double *l, const double *u) {
    if (q < 0 || q >= K) raise(PDLP_ERR_ARG, "instance index out of range");
    const int32_t c0 = h_col0[q], nq = h_col0[q + 1] - c0;
    if (nq == 0) return;
    if (!l || !u) raise(PDLP_ERR_ARG, "NULL bounds");
    std::vector<double> lh((size_t)nq), uh((size_t)nq);
    if (opt.device_ptrs) {
      HIPCHK(hipMemcpy(lh.data(), l, sizeof(double) * (size_t)nq, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(uh.data(), u, sizeof(double) * (size_t)nq, hipMemcpyDeviceToHost));
    } else {
      std::copy(l, l + nq, lh.begin());
      std::copy(u, u + nq, uh.begin());
    }
    std::vector<double> li((size_t)nq), ui((size_t)nq);
    for (int32_t j = 0; j < nq; ++j) {
      if (std::isnan(lh[j]) || std::isnan(uh[j])) raise(PDLP_ERR_ARG, "bounds must not be NaN");
      if (lh[j] > uh[j]) raise(PDLP_ERR_ARG, "l > u at column " + std::to_string(j));
      if (lh[j] == INFINITY || uh[j] == -INFINITY) raise(PDLP_ERR_ARG, "l = +inf or u = -inf");
      const int32_t ji = h_inv_c[(size_t)(c0 + j)] - c0;
      li[(size_t)ji] = lh[j], ui[(size_t)ji] = uh[j];
    }
    double *dl = mem.alloc<double>(nq), *du = mem.alloc<double>(nq);
    upload(dl, li.data(), nq);
    upload(du, ui.data(), nq);
    hipLaunchKernelGGL(k_scale_bounds<T>, dim3(grid_for(nq)), dim3(kBlock), 0, stream, nq, c0, (const double *)dl,
                       (const double *)du, (const double *)Dc, l64, u64, lT, uT);
    HIPCHK(hipGetLastError());
    sync();
    mem.release(dl), mem.release(du);
  }

  // Scaling in the caller's numbering: Dr [m], Dc [n], scaled values in the caller's CSR order.
  void get_scaling(double *dr, double *dc, double *sv) {
    std::vector<double> hr((size_t)m), hc((size_t)n), hv;
    download(hr.data(), Dr, m);
    download(hc.data(), Dc, n);
    if (sv) {
      hv.resize((size_t)nnz);
      download(hv.data(), a_v64, nnz);
    }
    sync();
    if (dr)
      for (int32_t e = 0; e < m; ++e) dr[e] = hr[h_inv_r[e]];
    if (dc)
      for (int32_t e = 0; e < n; ++e) dc[e] = hc[h_inv_c[e]];
    if (sv)
      for (int32_t k = 0; k < nnz; ++k) sv[k] = hv[h_nnz_map[k]];
  }

  // The internal (renumbered, scaled) matrix and its transpose as built on the device, with the
  // renumbering: internal row i is the caller's row row_perm[i], internal column j is col_perm[j].
  void get_internal(int32_t *rp, int32_t *ci, double *v, int32_t *trp, int32_t *tci, double *tv, int32_t *pr,
                    int32_t *pc) {
    if (rp) download(rp, a_rp, m + 1);
    if (ci) download(ci, a_ci, nnz);
    if (v) download(v, a_v64, nnz);
    if (trp) download(trp, t_rp, n + 1);
    if (tci) download(tci, t_ci, nnz);
    if (tv) download(tv, t_v64, nnz);
    sync();
    if (pr) std::copy(h_perm_r.begin(), h_perm_r.end(), pr);
    if (pc) std::copy(h_perm_c.begin(), h_perm_c.end(), pc);
  }
};

// Precision-erased handle.
struct AnySolver {
  std::unique_ptr<Solver<float>> f;
  std::unique_ptr<Solver<double>> d;
  template <typename F>
  void visit(F &&fn) {
    if (f) fn(*f);
    else fn(*d);
  }
  void create(const std::vector<const HostProblem *> &H, const pdlp_options &o) {
    if (o.precision == PDLP_FP64) {
      d = std::make_unique<Solver<double>>();
      d->create(H, o);
    } else {
      f = std::make_unique<Solver<float>>();
      f->create(H, o);
    }
  }
};

}  // namespace pdlp

// ================================================================================================
// extern "C" boundary
// ================================================================================================
struct pdlp_problem {
  pdlp::AnySolver s;
};
struct pdlp_batch {
  pdlp::AnySolver s;
  int32_t k = 0;
};

using pdlp::Error;

template <typename F>
static int guarded(F &&f) {
  try {
    f();
    return PDLP_OK;
  } catch (const Error &e) {
    pdlp::g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    pdlp::g_last_error = "host allocation failed";
    return PDLP_ERR_OOM;
  } catch (...) {
    pdlp::g_last_error = "unexpected C++ exception";
    return PDLP_ERR_HIP;
  }
}

static pdlp_options resolve_options(const pdlp_options *opt) {
  pdlp_options o;
  pdlp_options_default(&o);
  if (opt) o = *opt;
  if (o.eval_every <= 0) o.eval_every = 64;
  if (o.ruiz_iters < 0) pdlp::raise(PDLP_ERR_ARG, "ruiz_iters < 0");
  if (o.precision != PDLP_FP32 && o.precision != PDLP_FP64) pdlp::raise(PDLP_ERR_ARG, "unknown precision");
  return o;
}

static void fetch_host_problem(pdlp::HostProblem &H, int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, const double *val, const double *c, const double *b,
                               const char *sense, const double *l, const double *u, bool device) {
  using pdlp::raise;
  if (m < 0 || n < 0 || nnz < 0) raise(PDLP_ERR_ARG, "negative size");
  if (!row_ptr || (nnz > 0 && (!col_idx || !val)) || (n > 0 && (!c || !l || !u)) || (m > 0 && (!b || !sense)))
    raise(PDLP_ERR_ARG, "NULL data pointer");
  if (nnz >= (int64_t)INT32_MAX) raise(PDLP_ERR_ARG, "nnz must be below 2^31");
  H.m = m, H.n = n, H.nnz = nnz;
  H.rp.resize((size_t)m + 1), H.ci.resize((size_t)nnz), H.val.resize((size_t)nnz);
  H.c.resize((size_t)n), H.l.resize((size_t)n), H.u.resize((size_t)n), H.b.resize((size_t)m), H.sense.resize((size_t)m);
  auto cp = [&](void *dst, const void *src, size_t bytes) {
    if (!bytes) return;
    if (device) {
      hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
      if (e != hipSuccess) raise(PDLP_ERR_HIP, std::string("reading device input: ") + hipGetErrorString(e));
    } else {
      std::memcpy(dst, src, bytes);
    }
  };
  cp(H.rp.data(), row_ptr, sizeof(int32_t) * ((size_t)m + 1));
  cp(H.ci.data(), col_idx, sizeof(int32_t) * (size_t)nnz);
  cp(H.val.data(), val, sizeof(double) * (size_t)nnz);
  cp(H.c.data(), c, sizeof(double) * (size_t)n);
  cp(H.l.data(), l, sizeof(double) * (size_t)n);
  cp(H.u.data(), u, sizeof(double) * (size_t)n);
  cp(H.b.data(), b, sizeof(double) * (size_t)m);
  cp(H.sense.data(), sense, (size_t)m);
  pdlp::validate(H);
}

extern "C" {

void pdlp_options_default(pdlp_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = PDLP_FP32;
  o->eval_every = 64;
  o->ruiz_iters = 10;
  o->pock_chambolle = 1;
  o->use_graphs = 1;
  o->device_ptrs = 0;
  o->tile_nnz = 0;
  o->verbose = 0;
  o->device_mem_limit = 0;
  o->stream = nullptr;
  o->warm_fallback = 2;
  o->kernel_timing = 0;
}

const char *pdlp_error_string(int code) {
  switch (code) {
    case PDLP_OK: return "ok";
    case PDLP_ERR_ARG: return "invalid argument";
    case PDLP_ERR_CSR: return "malformed CSR matrix";
    case PDLP_ERR_OOM: return "out of device memory";
    case PDLP_ERR_HIP: return "HIP runtime error";
    case PDLP_ERR_STATE: return "call out of order";
    default: return "unknown error";
  }
}

const char *pdlp_last_error(void) { return pdlp::g_last_error.c_str(); }

int pdlp_create(pdlp_problem **out, int32_t m, int32_t n, int64_t nnz, const int32_t *row_ptr,
                const int32_t *col_idx, const double *val, const double *c, const double *b, const char *sense,
                const double *l, const double *u, const pdlp_options *opt) {
  if (!out) {
    pdlp::g_last_error = "out is NULL";
    return PDLP_ERR_ARG;
  }
  *out = nullptr;
  return guarded([&] {
    const pdlp_options o = resolve_options(opt);
    pdlp::HostProblem H;
    fetch_host_problem(H, m, n, nnz, row_ptr, col_idx, val, c, b, sense, l, u, o.device_ptrs != 0);
    auto p = std::make_unique<pdlp_problem>();
    p->s.create({&H}, o);
    *out = p.release();
  });
}

int pdlp_solve(pdlp_problem *p, double tol, int64_t iter_limit, const double *x0, const double *y0, double omega0) {
  if (!p || iter_limit <= 0 || std::isnan(tol) || std::isnan(omega0)) {
    pdlp::g_last_error = !p ? "NULL handle" : "iter_limit must be positive; tol / omega0 not NaN";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    const double *xs[1] = {x0}, *ys[1] = {y0};
    const double om[1] = {omega0};
    p->s.visit([&](auto &s) { s.solve(tol, iter_limit, xs, ys, om); });
  });
}

int pdlp_get(pdlp_problem *p, double *x, double *y, double *red_cost, pdlp_result *res) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { p->s.visit([&](auto &s) { s.get(0, x, y, red_cost, res); }); });
}

int pdlp_spmv(pdlp_problem *p, int32_t trans, const double *x, double *y) {
  if (!p || !x || !y || trans < 0 || trans > 3) {
    pdlp::g_last_error = "bad argument to pdlp_spmv";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { p->s.visit([&](auto &s) { s.spmv(trans, x, y); }); });
}

int pdlp_get_scaling(pdlp_problem *p, double *Dr, double *Dc, double *scaled_val) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { p->s.visit([&](auto &s) { s.get_scaling(Dr, Dc, scaled_val); }); });
}

int pdlp_get_internal(pdlp_problem *p, int32_t *row_ptr, int32_t *col, double *val, int32_t *t_row_ptr,
                      int32_t *t_col, double *t_val, int32_t *row_perm, int32_t *col_perm) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    p->s.visit([&](auto &s) { s.get_internal(row_ptr, col, val, t_row_ptr, t_col, t_val, row_perm, col_perm); });
  });
}

int pdlp_get_schedule(pdlp_problem *p, int32_t *tile_nnz, int32_t *tiles_a, int32_t *tiles_at) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    p->s.visit([&](auto &s) {
      if (tile_nnz) *tile_nnz = s.chunk_nnz;
      if (tiles_a) *tiles_a = s.a_nchunks;
      if (tiles_at) *tiles_at = s.t_nchunks;
    });
  });
}

int pdlp_kernel_stats(pdlp_problem *p, int32_t kernel, int64_t *launches, double *total_ms) {
  if (!p || kernel < 0 || kernel > 4) {
    pdlp::g_last_error = "bad argument to pdlp_kernel_stats";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    p->s.visit([&](auto &s) {
      if (launches) *launches = s.t_launches[kernel];
      if (total_ms) *total_ms = s.t_ms[kernel];
    });
  });
}

int64_t pdlp_device_bytes(const pdlp_problem *p) {
  if (!p) return 0;
  int64_t r = 0;
  const_cast<pdlp_problem *>(p)->s.visit([&](auto &s) { r = s.mem.used; });
  return r;
}

void pdlp_destroy(pdlp_problem *p) { delete p; }

int pdlp_batch_create(pdlp_batch **out, int32_t k, const pdlp_problem_desc *descs, const pdlp_options *opt) {
  if (!out || k <= 0 || !descs) {
    pdlp::g_last_error = "bad argument to pdlp_batch_create";
    return PDLP_ERR_ARG;
  }
  *out = nullptr;
  return guarded([&] {
    const pdlp_options o = resolve_options(opt);
    std::vector<pdlp::HostProblem> H((size_t)k);
    std::vector<const pdlp::HostProblem *> ptrs;
    for (int32_t q = 0; q < k; ++q) {
      const pdlp_problem_desc &d = descs[q];
      fetch_host_problem(H[q], d.m, d.n, d.nnz, d.row_ptr, d.col_idx, d.val, d.c, d.b, d.sense, d.l, d.u,
                         o.device_ptrs != 0);
      ptrs.push_back(&H[q]);
    }
    auto p = std::make_unique<pdlp_batch>();
    p->k = k;
    p->s.create(ptrs, o);
    *out = p.release();
  });
}

int pdlp_batch_solve(pdlp_batch *bt, double tol, int64_t iter_limit, const double *const *x0s,
                     const double *const *y0s, const double *omega0s) {
  if (!bt || iter_limit <= 0 || std::isnan(tol)) {
    pdlp::g_last_error = "bad argument to pdlp_batch_solve";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { bt->s.visit([&](auto &s) { s.solve(tol, iter_limit, x0s, y0s, omega0s); }); });
}

int pdlp_batch_get(pdlp_batch *bt, int32_t i, double *x, double *y, double *red_cost, pdlp_result *res) {
  if (!bt) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { bt->s.visit([&](auto &s) { s.get(i, x, y, red_cost, res); }); });
}

int pdlp_batch_get_schedule(pdlp_batch *bt, int32_t *tile_nnz, int32_t *tiles_a, int32_t *tiles_at) {
  if (!bt) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] {
    bt->s.visit([&](auto &s) {
      if (tile_nnz) *tile_nnz = s.chunk_nnz;
      if (tiles_a) *tiles_a = s.a_nchunks;
      if (tiles_at) *tiles_at = s.t_nchunks;
    });
  });
}

int pdlp_update_bounds(pdlp_problem *p, const double *l, const double *u) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { p->s.visit([&](auto &s) { s.update_bounds(0, l, u); }); });
}

int pdlp_batch_update_bounds(pdlp_batch *bt, int32_t i, const double *l, const double *u) {
  if (!bt) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { bt->s.visit([&](auto &s) { s.update_bounds(i, l, u); }); });
}

int pdlp_set_snapshots(pdlp_problem *p, int32_t k, double rel_tol) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { p->s.visit([&](auto &s) { s.set_snapshots(k, rel_tol); }); });
}

int pdlp_get_snapshots(pdlp_problem *p, int32_t cap, double *x, double *y, int64_t *attempt, double *rel_kkt,
                       int32_t *count) {
  if (!p) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { p->s.visit([&](auto &s) { s.get_snapshots(0, cap, x, y, attempt, rel_kkt, count); }); });
}

int pdlp_batch_set_snapshots(pdlp_batch *bt, int32_t k, double rel_tol) {
  if (!bt) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { bt->s.visit([&](auto &s) { s.set_snapshots(k, rel_tol); }); });
}

int pdlp_batch_get_snapshots(pdlp_batch *bt, int32_t i, int32_t cap, double *x, double *y, int64_t *attempt,
                             double *rel_kkt, int32_t *count) {
  if (!bt) {
    pdlp::g_last_error = "NULL handle";
    return PDLP_ERR_ARG;
  }
  return guarded([&] { bt->s.visit([&](auto &s) { s.get_snapshots(i, cap, x, y, attempt, rel_kkt, count); }); });
}

void pdlp_batch_destroy(pdlp_batch *bt) { delete bt; }

}  // extern "C"

#include "gnn_host.h"
#include "fix_host.h"
#include "prop_host.h"
