// Device kernels of reference snapshots: several LP reference solutions taken from one PDLP run.
//
// The paper's conclusion (section 5) proposes using the cycling convergence of PDLP to obtain several
// reference solutions for fix-and-propagate from one LP solve. The restarts of the method (the
// evaluation step of the restarted scheme, every eval_every attempts) mark where it leaves one
// cycle for the next, so a snapshot is a restart point: the candidate the solve restarts to (the
// current iterate or the average, whichever has the smaller weighted KKT error), taken when the
// relative KKT error the evaluation measured for it in the original space is at most rel_tol.
// Each instance keeps the newest K snapshots in a ring; the solve itself is not changed.
//
// k_snap_pick (one thread per instance, after k_eval_fin) decides and claims a ring slot;
// k_snap_copy (evaluation blocks, after k_restart) writes the restart point, unscaled
// (x = Dc x~, y = Dr y~), into that slot.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdlp_internal.h"

namespace pdlp {

struct Snap {
  int32_t K;          // ring slots per instance (>= 1)
  int32_t n, m;       // columns / rows of all instances (slot stride of x / y)
  double rel_tol;     // largest relative KKT error of a restart point that is kept
  double *x, *y;      // [K][n], [K][m] internal numbering, original space
  int64_t *attempt;   // [instances][K] attempt count at which the snapshot was taken
  double *rel;        // [instances][K] its relative KKT error as the evaluation measured it
  int32_t *taken;     // [instances] snapshots taken since the solve started
  int32_t *slot;      // [instances] slot claimed at the last evaluation, -1 for none
};

__global__ __launch_bounds__(kBlock) void k_snap_pick(int ninst, const State *__restrict__ sts, Snap S) {
  const int q = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (q >= ninst) return;
  const State *st = sts + q;
  int s = -1;
  if (!st->done && st->restart_mode != kNoRestart) {
    const double rel = st->cand_rel[st->restart_mode == kToAverage ? 1 : 0];
    if (rel <= S.rel_tol) {
      const int t = S.taken[q];
      s = t % S.K;
      S.attempt[(size_t)q * S.K + s] = st->k;
      S.rel[(size_t)q * S.K + s] = rel;
      S.taken[q] = t + 1;
    }
  }
  S.slot[q] = s;
}

// After k_restart the committed iterate x[cur], y[cur] is the restart point (in FP32 the average
// enters it rounded to FP32, and the snapshot is that point, the one the method continues from).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_snap_copy(Iter<T> P, Snap S) {
  const int inst = P.L.ev_inst[blockIdx.x];
  const int s = S.slot[inst];
  if (s < 0) return;
  const int b0 = P.L.ev_blk0[inst], nlb = P.L.ev_blk0[inst + 1] - b0, lb = (int)blockIdx.x - b0;
  const int cur = P.st[inst].cur;
  const T *__restrict__ x = P.x[cur];
  const T *__restrict__ y = P.y[cur];
  double *__restrict__ xs = S.x + (size_t)s * (size_t)S.n;
  double *__restrict__ ys = S.y + (size_t)s * (size_t)S.m;
  const int gs = nlb * kBlock, off = lb * kBlock + (int)threadIdx.x;
  for (int j = P.L.col0[inst] + off; j < P.L.col0[inst + 1]; j += gs) xs[j] = P.Dc[j] * double(x[j]);
  for (int i = P.L.row0[inst] + off; i < P.L.row0[inst + 1]; i += gs) ys[i] = P.Dr[i] * double(y[i]);
}

}  // namespace pdlp
