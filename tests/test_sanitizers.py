"""The C oracles under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

A small driver program includes both oracle sources and runs every entry point (scaling, transpose,
product, one PDHG step, a solve with a trace, the KKT evaluation, propagation to a fixpoint and to
infeasibility) on a 3 x 4 LP with free, boxed and one-sided columns. Built with gcc and
-fsanitize=address,undefined (host code only; nothing runs on a GPU), it must exit cleanly with no
sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include "pdhg_oracle.c"
#include "prop_oracle.c"

int main(void) {
  /* rows: x0 + 2 x1 - x3 <= 4 ; x1 + x2 >= 1 ; x0 - x2 + x3 = 2 */
  const int32_t rp[4] = {0, 3, 5, 8};
  const int32_t ci[8] = {0, 1, 3, 1, 2, 0, 2, 3};
  const double v[8] = {1, 2, -1, 1, 1, 1, -1, 1};
  const double c[4] = {1, -1, 0.5, 2}, b[3] = {4, 1, 2};
  const uint8_t sense[3] = {'L', 'G', 'E'};
  double l[4] = {0, -INFINITY, 0, -2}, u[4] = {5, 3, INFINITY, INFINITY};
  orc_lp lp = {3, 4, rp, ci, v, c, b, sense, l, u};
  double Dr[3], Dc[4], sv[8], y[3], ax[3], x[4] = {1, 0.5, 0.5, 1}, xn[4], yn[3];
  int32_t trp[5], tci[8];
  double tv[8];
  if (orc_scale(3, 4, rp, ci, v, 10, 1, Dr, Dc, sv) != 0) return 1;
  orc_transpose(3, 4, rp, ci, v, trp, tci, tv);
  orc_spmv(3, rp, ci, v, x, ax);
  y[0] = -0.5, y[1] = 0.25, y[2] = 1.0;
  if (orc_pdhg_step(&lp, x, y, 0.1, 0.1, xn, yn) != 0) return 2;
  enum { K = 40 };
  static double tx[K * 4], ty[K * 3], te[K], tw[K], tm[K], tc[K];
  static int32_t tf[K];
  orc_opts o = {1e-6, 5000, 10, 1, 64, K, NULL, NULL, 0.0, tx, ty, te, tw, tf, tm, tc};
  double xs[4], ys[3], rc[4], kk[7];
  orc_result r;
  if (orc_solve(&lp, &o, xs, ys, rc, &r) != 0) return 3;
  if (orc_kkt(&lp, xs, ys, kk) != 0) return 4;
  const uint8_t vt[4] = {2, 1, 0, 2};
  double pl[4] = {0, 0, 0, -2}, pu[4] = {5, 1, 10, 4};
  int32_t rounds = 0;
  int st = orc_propagate(3, 4, rp, ci, v, b, sense, vt, pl, pu, 50, &rounds);
  double ql[4] = {0, 0, 0, 3}, qu[4] = {0, 0, 0, 3};
  int st2 = orc_propagate(3, 4, rp, ci, v, b, sense, vt, ql, qu, 50, &rounds);
  printf("solve status %d iterations %lld rel_kkt %.2e; propagation %d then %d\n", r.status,
         (long long)r.iterations, fmax(r.rel_p, fmax(r.rel_d, r.rel_gap)), st, st2);
  return (r.status == 1 && st == 0 && st2 == 1) ? 0 : 5;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracles_clean_under_asan_and_ubsan(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=gnu99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"), str(src),
           "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtime not installed")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    print(run.stdout, run.stderr)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
