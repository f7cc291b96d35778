// Internal declarations shared by the HIP kernels and the host runtime of libpdlp.
//
// One handle solves K >= 1 independent LPs. Their matrices are stored as one block-diagonal CSR
// (and its transpose) with global row/column indices; every launch covers all instances, and each
// block looks up the instance it works for. A single-LP handle is the case K = 1.
//
// Inside a handle the rows and the columns of every instance are renumbered so that rows of A and
// rows of A' (columns of A) come sorted by length class (stable within a class). Every vector on
// the device is in this internal order; inputs and outputs are mapped at the boundary.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdlp {

constexpr int kBlock = 256;   // threads per block for every kernel
constexpr int kWave = 64;     // CDNA wavefront
constexpr int kWaves = kBlock / kWave;
constexpr int kEvalNV = 18;   // per-block partial sums of the evaluation kernel
constexpr int kEvalSpan = 2048;    // elements per evaluation block (target)
// Column-panel path of A x for long rows (FP32): x is cut into panels of kPanelW entries that a
// work group keeps in LDS while it sums its rows' entries in that panel; the per-panel sums of a
// row (FP64) are added up in panel order by the kernel that runs the row's epilogue.
constexpr int kPanelW = 16384;     // x entries per panel (64 KB of FP32 in LDS)
constexpr int kPanelBlock = 1024;  // threads per panel work group
// Column-block path of A'y (FP32): a work group owns kCbCols consecutive columns and reads y in row
// panels of kCbRows entries held in LDS; see ColBlocks.
constexpr int kCbCols = 4096;      // columns per work group
constexpr int kCbRows = 16384;     // y entries per panel (64 KB of FP32)
constexpr int kCbBlock = 1024;     // threads per work group
constexpr int kCbMaxPanels = 512;  // instances with more y panels keep the chunk engine
constexpr int kCbMaxGroups = 4096; // work groups with more run groups than this keep the chunk engine

enum RestartMode : int32_t { kNoRestart = 0, kToCurrent = 1, kToAverage = 2 };
enum EvalMode : int32_t { kEvalInit = 0, kEvalChunk = 1, kEvalPoint = 2 };
// What k_primal does to the running averages on an accepted attempt. With paired updates (FP32),
// every other accepted attempt leaves its update pending and the next one applies both in one pass
// over x-bar and y-bar (the older iterate is still in the other buffer then); the operations and
// their order are those of two single updates, so the averages are bitwise the same.
enum AvgMode : int32_t { kAvgOne = 0, kAvgDefer = 1, kAvgPair = 2 };

// Per-instance solver state on the device. Written only by the last block of an instance in a
// kernel (or by the host between solves); read by every block of that instance at kernel start.
struct State {
  double eta;         // step size of the next attempt (scaled space)
  double omega;       // primal weight
  double wsum;        // sum of accepted step sizes since the last restart
  double avg_w;       // weight eta/wsum of the newest accepted attempt's average update
  double avg_w1;      // paired update: weight of the older accepted attempt (applied first)
  double pend_w;      // paired updates: weight of an accepted attempt whose update waits (0: none)
  double dx2;         // |x' - x|^2 of the pending primal candidate
  double kkt_anchor;  // weighted KKT error of the last restart point
  double kkt_prev;    // weighted KKT error of the previous restart candidate
  double tol;         // relative KKT tolerance (<= 0: never met)
  double rel_p, rel_d, rel_gap, pobj, dobj;  // last evaluated point (original space)
  double cand_rel[2]; // relative KKT error of current [0] / average [1] at the last evaluation
  double ev_rel[6];   // at the last evaluation: rel_p, rel_d, rel_gap of current [0..2] and average [3..5]
  double nb, nc;      // |b|, |c| of the original data
  int64_t k;          // attempts so far
  int64_t last_restart;
  int64_t iter_limit;
  int32_t cur;        // which buffer of x/y/ax holds the committed iterate
  int32_t commit;     // 1: the last attempt was accepted and awaits the transposed product
  int32_t stop;       // 1: finish after the pending commit / restart
  int32_t done;       // 1: no further work
  int32_t status;     // PDLP_STATUS_*
  int32_t which;      // returned point: 0 current, 1 average
  int32_t restarts;
  int32_t restart_mode;
  int32_t eval_every;
  int32_t avg_mode;   // AvgMode of the last accepted attempt
  int32_t pair_avg;   // 1: pair the average updates of consecutive accepted attempts
  int32_t pad_;
};

// Instance layout tables (device arrays).
struct Layout {
  int32_t K;
  const int32_t *row0, *col0;       // [K+1] row / column offsets
  const int32_t *a_chunk0, *t_chunk0; // [K+1] chunk ranges of A and A'
  const int32_t *ab0, *ab_inst;     // [K+1], [ab_blocks] A-side work blocks (k_dual)
  const int32_t *tb0, *tb_inst;     // [K+1], [tb_blocks] A'-side work blocks (k_primal)
  const int32_t *a_bchunk;           // [2 ab_blocks] first and end chunk of each A-side work block;
                                     // (-1 - j, -1 - j) for long-row block j (no chunks)
  const int32_t *t_bchunk;           // [tb_blocks + 1] first chunk of each A'-side work block
  const int32_t *ev_blk0, *ev_inst; // [K+1], [ev_blocks] evaluation blocks
  int32_t a_nchunks, t_nchunks, ab_blocks, tb_blocks, ev_blocks;
  // long rows of A (column-panel path): the first lr_R[q] rows of instance q; their panel sums are
  // part[lr_base[q] + p * lr_R[q] + r], p < lr_P[q]; long-row block j of the instance's A-side
  // blocks finishes its rows [kBlock j, kBlock (j + 1)). All zero without the path.
  const int32_t *lr_R, *lr_P;
  const int64_t *lr_base;
  // A' side: instance q's |dx|^2 partials are p_primal[pb0[q] .. pb0[q+1]); cb_n[q] > 0 when its A'y
  // runs by column blocks (that many work groups of k_primal_cb; k_primal skips the instance).
  const int32_t *pb0, *cb_n;
  // A side: instance q's (|dy|^2, dy'(A dx)) partial pairs are p_dual[2 (db0[q] .. db0[q+1])); rb_n[q]
  // > 0 when its A x runs by row blocks (that many work groups of k_dual_rb; k_dual skips it).
  const int32_t *db0, *rb_n;
  // Per launch block of k_dual (ab_blocks) and of k_primal (tb_blocks), everything the block needs
  // to start, with the XCD remapping applied: (instance, first chunk, end chunk, partial slot), and
  // for k_primal its share (first, end) of the instance's rows. A long-row block of k_dual has the
  // chunk pair (-1 - j, -1 - j).
  const int4 *ia_desc, *tb_desc;
  const int2 *tb_rows;
};

// Column-panel work groups: (row block, panel) pairs. A row block is a run of consecutive long rows
// of one instance; its entries in panel p are stored row by row (each row's in CSR order) as a
// 16-bit column offset within the panel and a value, with per-row start offsets (16-bit, relative
// to the work group's first entry).
template <typename T>
struct Panels {
  int32_t nwg;
  const int32_t *wg_rb, *wg_p;      // [nwg] row block and panel of each work group
  const int64_t *wg_ebase;          // [nwg] first entry of the work group
  const int64_t *wg_obase;          // [nwg] first of its R + 1 row offsets
  const int32_t *rb_inst, *rb_lrow0, *rb_R, *rb_G;  // row block: instance, first long row (index
                                    // within the instance), rows, lanes per row
  const uint16_t *off, *col;
  const T *val;
};

// Column blocks of A' (rows of A' = columns of A). Work group w owns the columns
// [col0[q] + kCbCols * wg_blk[w], ...) of instance q = wg_inst[w]. The first ndense[q] row panels
// of kCbRows rows (the dense ones: rows are stored longest first) are read through LDS; the
// entries in later rows (the tail) gather y directly.
// Panels: in panel p a column's entries form a run (in row order); the work group's runs in panel
// p are sorted by length (longest first) and dealt to groups of 64 lanes, the groups
// [gstart[wg_g0[w] + p], gstart[wg_g0[w] + p + 1]). Group g: desc[64 g + l] = (length << 16) |
// (column within the block) of lane l's run, 0 for a lane without one; entry t of lane l's run is
// at index 64 (ebase[g] + t) + l of row (row within the panel) and val, for t below the group's
// longest run (lane 0's). Slots past a run's end hold row 0 and value 0, and the entry arrays end
// with one spare slot of 64 entries, so a group's second slot can always be read.
// Tail: a column's tail entries form one run; the work group's tail runs, sorted by length, are
// dealt to the groups [wg_t[w], wg_t[w + 1]), laid out as above in tdesc, tebase (one entry past
// the last group too), trow (row within the instance) and tval.
template <typename T>
struct ColBlocks {
  int32_t nwg;
  const int32_t *ndense;
  const int32_t *wg_inst, *wg_blk, *wg_g0;
  const int32_t *gstart;
  const uint32_t *desc;
  const int32_t *ebase;
  const uint16_t *row;
  const T *val;
  const int32_t *wg_t;
  const uint32_t *tdesc;
  const int32_t *tebase;
  const int32_t *trow;
  const T *tval;
};

// Everything an iteration kernel reads or writes. Passed by value.
template <typename T>
struct Iter {
  Layout L;
  // A (row view) and A' (column view), scaled, in the iteration precision, rows sorted by length
  // class; chunk_row[k] is the first row of chunk k and chunk_cls[k] its class
  const int32_t *a_rp, *a_ci, *a_chunk_row;
  const int8_t *a_chunk_cls;
  const T *a_val;
  const int32_t *t_rp, *t_ci, *t_chunk_row;
  const int8_t *t_chunk_cls;
  const T *t_val;
  // problem data, scaled
  const T *c, *l, *u, *b;
  const uint8_t *sense;
  const double *Dr, *Dc;
  // iterates
  T *x[2], *y[2], *ax[2];
  T *aty;
  double *xbar, *ybar;  // running averages: FP64 in both precisions (FP32 would lose late updates)
  T *axbar, *atybar;
  T *xa, *ya;
  // block partial sums (one slot per block of the producing kernel) and state
  double *p_dual;     // [ab_blocks][2]  |dy|^2, dy'(A dx)
  double *p_primal;   // [tb_blocks]     |dx|^2 of the primal candidate
  double *p_restart;  // [ev_blocks]     |dx|^2 after a restart
  double *p_eval;     // [ev_blocks][kEvalNV]
  double *part;       // panel sums of the long rows (see Layout)
  State *st;
  int32_t *ndone;  // number of instances with done == 1
};

}  // namespace pdlp
