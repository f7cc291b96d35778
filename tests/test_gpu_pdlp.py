"""GPU parity tests: the HIP path through the C-ABI against the FP64 oracle (and HiGHS / scipy).

Tolerances:
  * SpMV, FP64: |y - y_ref| <= 1e-12 (|A||x|)_i ; FP32: <= 2e-6 (|A||x|)_i + 1e-30 (the inputs are
    rounded to FP32 once, each product and sum adds one rounding; sqrt(5000) * 2^-24 < 5e-6 for the
    longest rows, far below what accumulates in practice).
  * Scaling (FP64 on the GPU): Dr, Dc and the scaled values within 1e-12 relative of the oracle; the
    sums of the Pock-Chambolle pass are taken in a different order, so bitwise equality is not
    expected.
  * Transpose: bit-exact (integer work; the values are gathered, not computed).
  * Iterate tracking (FP64): |x_k^gpu - x_k^orc| <= B_k |x_k^orc| (likewise y and omega) for
    k = 1..100 with B_k = max(1e-9, 2 D_k), where D_k is the running maximum of how far the oracle's
    own iterates move when every sum is taken in another order (reversed; even indices first): the
    method amplifies rounding differences by ~15 % per attempt on degenerate LPs, and D_k passes
    1e-9 near k = 90 on the set-cover and energy cases (tests/tracking.py). Attempts after a discrete
    decision with relative margin < 1e-12 are not compared. The step size eta is a ratio of squared
    step lengths |dx|^2, |dy|^2: a relative error e of the iterates enters it as e |x| / |dx| (and
    e |y| / |dy|), so its bound is B_k times the largest such factor the oracle recorded up to k.
  * End to end: relative KKT <= tol as re-evaluated by the oracle from the returned point. The
    objective: within 1e-4 relative (max(1, |f|)) of the oracle solved to the same tolerance where
    the oracle converges quickly, and always inside the interval LP duality gives for a point with
    the returned residuals: -|y*| |r_p| <= c'x - f* <= (pobj - dobj) + |x*| |r_d| (x*, y* from
    HiGHS, residuals re-evaluated by the oracle). A relative KKT error of 1e-4 does not by itself
    bound the objective error by 1e-4: the primal residual is normalised by |b|.
"""
import sys

import numpy as np
import pytest

import oracle
import oracle_pins as P
import tracking

try:  # import at collection time: the first import on a fresh machine can take a minute
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None
from paper_2503_10344_amd import generators as g

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pdlp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_10344_amd import pdlp as mod
    mod.load()
    return mod


def _objective_interval_ok(lp, sol_x, sol_y, f, xs, ys, label=""):
    """c'x - f* inside the interval weak duality gives for the returned residuals (see above)."""
    k = oracle.kkt(lp, sol_x, sol_y)
    lo = -np.linalg.norm(ys) * k["norm_rp"]
    hi = (k["pobj"] - k["dobj"]) + np.linalg.norm(xs) * k["norm_rd"]
    d = k["pobj"] - f
    slack = 1e-9 * max(1.0, abs(f))
    say(label, "objective error %.3e in [%.3e, %.3e]; rel %.2e" % (d, lo, hi, abs(d) / max(1.0, abs(f))))
    assert lo - slack <= d <= hi + slack, (d, lo, hi)
    return k


def _absprod(lp, x):
    A = lp.to_scipy()
    return abs(A) @ np.abs(x)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spmv_parity(pdlp, prec):
    lp = g.general_sparse(1, m=20000, n=40000)  # rows up to 5000 long: stream and long tiles
    say("spmv", prec, lp.m, lp.n, lp.nnz)
    A = lp.to_scipy()
    rng = np.random.default_rng(2)
    x = rng.standard_normal(lp.n)
    y = rng.standard_normal(lp.m)
    tol = 1e-12 if prec == "fp64" else 2e-6
    for tn in (512, 2048, 4096):
        with pdlp.Problem(lp, precision=prec, tile_nnz=tn) as p:
            ax = p.spmv(x)
            aty = p.spmv(y, trans=True)
        ref = oracle.spmv(lp.row_ptr, lp.col, lp.val, x)
        assert np.all(np.abs(ax - ref) <= tol * _absprod(lp, x) + 1e-30), (tn, np.abs(ax - ref).max())
        refT = A.T @ y
        bound = abs(A).T @ np.abs(y)
        assert np.all(np.abs(aty - refT) <= tol * bound + 1e-30), (tn, np.abs(aty - refT).max())


def test_spmv_edge_shapes(pdlp):
    # empty rows, empty columns, a single dense row, and a ragged tail
    rng = np.random.default_rng(5)
    m, n = 1500, 3000
    rows, cols, vals = [], [], []
    for i in range(m):
        if i % 7 == 0:
            continue  # empty row
        L = 4100 if i == 700 else int(rng.integers(1, 40))
        cs = np.sort(rng.choice(n - 50, size=min(L, n - 50), replace=False))  # last 50 columns empty
        rows += [i] * cs.size
        cols += cs.tolist()
        vals += rng.standard_normal(cs.size).tolist()
    rp, ci, v = g._csr_from_triplets(m, n, rows, cols, vals)
    lp = g.LP(m, n, rp, ci, v, np.zeros(n), np.zeros(m), np.full(m, ord("E"), np.uint8),
              np.full(n, -np.inf), np.full(n, np.inf))
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    A = lp.to_scipy()
    for prec, tol in (("fp64", 1e-12), ("fp32", 2e-6)):
        with pdlp.Problem(lp, precision=prec, tile_nnz=1024) as p:
            ax, aty = p.spmv(x), p.spmv(y, trans=True)
        assert np.all(np.abs(ax - A @ x) <= tol * (abs(A) @ np.abs(x)) + 1e-30)
        assert np.all(np.abs(aty - A.T @ y) <= tol * (abs(A).T @ np.abs(y)) + 1e-30)
        assert np.all(ax[::7] == 0.0) and np.all(aty[-50:] == 0.0)


def test_long_rows_block_path_is_bitwise_the_wave_path(pdlp):
    """Rows of >= 1024 nonzeros alone in a chunk are summed by a whole block; the sum must be
    bitwise the one wave computes when the same row shares a chunk with others (larger chunks)."""
    rng = np.random.default_rng(11)
    m, n = 2000, 8000
    rows, cols, vals = [], [], []
    for i in range(m):
        L = int(rng.choice([1100, 1300, 1500, 1800, 2900])) if i % 5 == 0 else int(rng.integers(1, 60))
        cs = np.union1d(np.arange(10), rng.choice(np.arange(10, n), size=L, replace=False))  # 10 dense columns
        rows += [i] * cs.size
        cols += cs.tolist()
        vals += rng.standard_normal(cs.size).tolist()
    rp, ci, v = g._csr_from_triplets(m, n, rows, cols, vals)
    lp = g.LP(m, n, rp, ci, v, np.zeros(n), np.zeros(m), np.full(m, ord("E"), np.uint8),
              np.full(n, -np.inf), np.full(n, np.inf))
    x = rng.standard_normal(n)
    y = rng.standard_normal(m)
    for prec in ("fp32", "fp64"):
        out = {}
        for cap in (512, 4096):
            with pdlp.Problem(lp, precision=prec, tile_nnz=cap) as p:
                out[cap] = (p.spmv(x), p.spmv(y, trans=True))
        np.testing.assert_array_equal(out[512][0], out[4096][0])
        np.testing.assert_array_equal(out[512][1], out[4096][1])


def test_transpose_and_scaling(pdlp):
    lp = g.general_sparse(3, m=4000, n=9000, cap=2000)
    say("scaling", lp.m, lp.n, lp.nnz)
    with pdlp.Problem(lp, precision="fp64") as p:
        s = p.scaling()
        it = p.internal()
    Dr, Dc, sv = oracle.scale(lp)
    assert np.allclose(s["Dr"], Dr, rtol=1e-12, atol=0) and np.allclose(s["Dc"], Dc, rtol=1e-12, atol=0)
    assert np.allclose(s["scaled_val"], sv, rtol=1e-12, atol=0)
    # the internal numbering is a permutation sorting rows / columns by length class
    pr, pc = it["row_perm"], it["col_perm"]
    assert np.array_equal(np.sort(pr), np.arange(lp.m)) and np.array_equal(np.sort(pc), np.arange(lp.n))
    rlen = np.diff(lp.row_ptr)[pr]
    cls = np.where(rlen <= 3, 0, np.minimum(6, np.floor(np.log2(np.maximum(rlen, 1))).astype(int) - 1))
    assert np.all(np.diff(cls) <= 0)
    # internal A is the caller's A with rows and columns renumbered, values scaled
    A = lp.to_scipy()
    Ai = __import__("scipy.sparse", fromlist=["csr_matrix"]).csr_matrix(
        (it["val"], it["col"], it["row_ptr"]), shape=(lp.m, lp.n))
    S = (A.multiply(Dr[:, None]).multiply(Dc[None, :])).tocsr()[pr][:, pc]
    assert abs(Ai - S).max() <= 1e-12 * abs(S).max()
    # the transpose built on the device is bit-exact against the oracle's counting sort
    trp, tci, tv = oracle.transpose(lp.m, lp.n, it["row_ptr"], it["col"], it["val"])
    assert np.array_equal(it["t_row_ptr"], trp) and np.array_equal(it["t_col"], tci)
    assert np.array_equal(it["t_val"], tv)  # gathered, so bitwise equal to the row copy


def _tracking(pdlp, lp, K=100, label=""):
    orc = oracle.solve(lp, tol=0.0, iter_limit=K, trace_len=K)
    tr = orc.trace
    cut = K
    bad = np.nonzero(tr["margin"] < 1e-12)[0]
    if bad.size:
        cut = int(bad[0])  # compare only before the first near-tie
        say(label, "near-tie at attempt", cut + 1, "- comparing attempts 1 ..", cut)
    bound = tracking.tracking_bound(lp, K, tr)
    ks = list(range(1, cut + 1))
    worst, worst_ratio = 0.0, 0.0
    with pdlp.Problem(lp, precision="fp64", tile_nnz=1024, warm_fallback=False) as p:
        for k in ks:
            p.solve(tol=0.0, iter_limit=k)
            sol = p.get()
            xo, yo = tr["x"][k - 1], tr["y"][k - 1]
            ex = np.linalg.norm(sol.x - xo) / max(np.linalg.norm(xo), 1e-30)
            ey = np.linalg.norm(sol.y - yo) / max(np.linalg.norm(yo), 1e-30)
            eeta = abs(sol.info["eta"] - tr["eta"][k - 1]) / tr["eta"][k - 1]
            eom = abs(sol.info["omega"] - tr["omega"][k - 1]) / tr["omega"][k - 1]
            cond = float(tr["cond"][:k].max())
            assert sol.info["iterations"] == k
            b = bound[k - 1]
            say(label, "k", k, "err x %.2e y %.2e omega %.2e eta %.2e bound %.2e" % (ex, ey, eom, eeta, b))
            assert max(ex, ey, eom) <= b, (label, k, ex, ey, eom, b)
            assert eeta <= b * cond, (label, k, eeta, cond, b)
            worst = max(worst, ex, ey, eom)
            worst_ratio = max(worst_ratio, max(ex, ey, eom) / b)
    flags = tr["flags"][:cut]
    say(label, "tracked", cut, "attempts; accepted", int((flags & 1).sum()), "restarts",
        int(((flags & 4) > 0).sum()), "worst iterate rel err %.2e (%.2f of the bound); bound at %d: %.2e"
        % (worst, worst_ratio, cut, bound[cut - 1]))


def test_tracking_fp64_setcover(pdlp):
    _tracking(pdlp, g.set_cover(0, m=300, n=700), label="setcover")


def test_tracking_fp64_general(pdlp):
    _tracking(pdlp, g.general_sparse(2, m=400, n=800, cap=200), label="general")


def test_tracking_fp64_energy(pdlp):
    _tracking(pdlp, g.energy(1, T=24, N=5, K=3, E=8), label="energy")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_end_to_end_setcover(pdlp, prec):
    lp = g.set_cover(0)  # 2000 x 5000, the correctness / latency workload
    f, xs, ys = P.highs(lp)
    orc = oracle.solve(lp, tol=1e-4)
    with pdlp.Problem(lp, precision=prec) as p:
        info = p.solve(tol=1e-4)
        sol = p.get()
    say("setcover", prec, info["status_name"], info["iterations"], info["primal_obj"], "oracle", orc.pobj, "highs", f)
    assert info["status"] == pdlp.OPTIMAL
    k = _objective_interval_ok(lp, sol.x, sol.y, f, xs, ys, "setcover")
    assert k["rel_kkt"] <= 1e-4, k
    assert abs(info["primal_obj"] - orc.pobj) <= 1e-4 * max(1.0, abs(orc.pobj))
    assert abs(k["pobj"] - info["primal_obj"]) <= 1e-9 * max(1.0, abs(f))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_setcover_seeds_reach_tolerance(pdlp, prec):
    """Set cover 2,000 x 5,000, seeds 0-9 (the small-LP latency workload): every solve ends optimal
    with the oracle's relative KKT error of the returned point at most 1e-4."""
    worst = 0.0
    for seed in range(10):
        lp = g.set_cover(seed)
        with pdlp.Problem(lp, precision=prec) as p:
            info = p.solve(tol=1e-4, iter_limit=100_000)
            sol = p.get()
        k = oracle.kkt(lp, sol.x, sol.y)
        worst = max(worst, k["rel_kkt"])
        assert info["status"] == pdlp.OPTIMAL and k["rel_kkt"] <= 1e-4, (seed, info["iterations"], k["rel_kkt"])
    say("setcover seeds 0-9", prec, "worst oracle rel_kkt %.3e" % worst)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_end_to_end_energy(pdlp, prec):
    lp = g.energy(4, T=96, N=8, K=6, E=16)
    f, xs, ys = P.highs(lp)
    orc = oracle.solve(lp, tol=1e-4)
    with pdlp.Problem(lp, precision=prec) as p:
        info = p.solve(tol=1e-4, iter_limit=400_000)
        sol = p.get()
    say("energy", prec, info["status_name"], info["iterations"], info["primal_obj"], "oracle", orc.pobj,
        orc.iterations, "highs", f)
    assert info["status"] == pdlp.OPTIMAL
    assert _objective_interval_ok(lp, sol.x, sol.y, f, xs, ys, "energy")["rel_kkt"] <= 1e-4
    assert abs(info["primal_obj"] - orc.pobj) <= 1e-4 * max(1.0, abs(orc.pobj))


@pytest.fixture(scope="module")
def general7():
    """The 3,000 x 6,000 general sparse LP (seed 7), its HiGHS optimum and the oracle at 1e-4."""
    lp = g.general_sparse(7, m=3000, n=6000, cap=1000)
    f, xs, ys = P.highs(lp)
    return lp, f, xs, ys, oracle.solve(lp, tol=1e-4, iter_limit=400_000)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_end_to_end_general(pdlp, prec, general7):
    """Relative KKT 1e-4 as the oracle re-evaluates it, and the objective inside the weak-duality
    interval around HiGHS's optimum. Neither the attempt count nor the objective at 1e-4 is compared
    with the oracle's: any rounding difference changes a restart decision after a few thousand
    attempts (the oracle's own summation orders part at attempt 5,696 on this LP and stop at 32,256
    to 36,352 attempts), and 1e-4 points of this LP differ by ~1e-3 relative in objective
    (||x*|| ~ 9e5, so small relative infeasibility moves c'x). Both are printed."""
    lp, f, xs, ys, orc = general7
    with pdlp.Problem(lp, precision=prec) as p:
        info = p.solve(tol=1e-4, iter_limit=2_000_000)
        sol = p.get()
    say("general", prec, info["status_name"], info["iterations"], info["primal_obj"], "oracle", orc.pobj,
        orc.iterations, "highs", f, "rel to oracle %.2e" % (abs(info["primal_obj"] - orc.pobj) / abs(orc.pobj)))
    assert info["status"] == pdlp.OPTIMAL and orc.status == oracle.OPTIMAL
    assert _objective_interval_ok(lp, sol.x, sol.y, f, xs, ys, "general")["rel_kkt"] <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tighter_tolerance_gives_the_objective_within_1e4_of_the_optimum(pdlp, prec, general7):
    """Objective accuracy is a matter of tolerance: solved to relative KKT 3e-5, the general LP's
    objective lies within 1e-4 relative of HiGHS's optimum in both precisions (at 1e-4 it is
    ~1.2e-3 away)."""
    lp, f, xs, ys, _ = general7
    with pdlp.Problem(lp, precision=prec) as p:
        info = p.solve(tol=3e-5, iter_limit=2_000_000)
        sol = p.get()
    k = oracle.kkt(lp, sol.x, sol.y)
    say("general tol 3e-5", prec, info["status_name"], info["iterations"], info["primal_obj"], "highs", f,
        "rel err %.2e" % (abs(info["primal_obj"] - f) / abs(f)), "oracle rel_kkt %.2e" % k["rel_kkt"])
    assert info["status"] == pdlp.OPTIMAL and k["rel_kkt"] <= 3e-5
    assert abs(info["primal_obj"] - f) <= 1e-4 * max(1.0, abs(f))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reduced_costs_match_the_oracle(pdlp, prec, general7):
    """pdlp_get's reduced costs are c - A'y of the returned y (FP64 from the FP64 matrix in both
    precisions): against the oracle's product on the caller's data, every entry within 1e-12 of
    |c_j| + (|A|'|y|)_j, on LPs with rows of every sense and free, boxed and one-sided columns."""
    lps = [general7[0], g.set_cover(0), g.energy(4, T=96, N=8, K=6, E=16), g.multi_knapsack(1, m=150, n=400)]
    for lp in lps:
        with pdlp.Problem(lp, precision=prec) as p:
            p.solve(tol=1e-4, iter_limit=1_000_000)
            sol = p.get()
        trp, tci, tv = oracle.transpose(lp.m, lp.n, lp.row_ptr, lp.col, lp.val)
        rc = lp.c - oracle.spmv(trp, tci, tv, sol.y)
        scale = np.abs(lp.c) + oracle.spmv(trp, tci, np.abs(tv), np.abs(sol.y))
        err = np.max(np.abs(sol.rc - rc) / np.maximum(scale, 1e-300))
        say("reduced costs", prec, lp.name, "max rel err %.2e" % err)
        assert np.all(np.abs(sol.rc - rc) <= 1e-12 * scale + 1e-300)


def test_fp64_matches_oracle_iterations(pdlp):
    """FP64 GPU solve to 1e-6 against the oracle's: same status, iteration counts within 30 % (the
    two differ only in rounding order, which the method amplifies; the stopping evaluation can move
    by a few intervals), objectives within the 2 tol band the gap test allows each of them."""
    lp = g.set_cover(4, m=500, n=1200)
    orc = oracle.solve(lp, tol=1e-6)
    with pdlp.Problem(lp, precision="fp64") as p:
        info = p.solve(tol=1e-6)
    say("fp64 vs oracle", info["iterations"], orc.iterations, info["primal_obj"], orc.pobj)
    assert info["status"] == pdlp.OPTIMAL and orc.status == oracle.OPTIMAL
    assert abs(info["iterations"] - orc.iterations) <= max(128, 0.3 * orc.iterations)
    assert abs(info["primal_obj"] - orc.pobj) <= 4e-6 * max(1.0, abs(orc.pobj))


def test_determinism(pdlp):
    lp = g.general_sparse(7, m=2000, n=4000, cap=800)
    with pdlp.Problem(lp, precision="fp32") as p:
        p.solve(tol=1e-4)
        a = p.get()
        p.solve(tol=1e-4)
        b = p.get()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)
    assert a.info["iterations"] == b.info["iterations"]


def test_paired_average_updates_are_bitwise_single_updates(pdlp):
    """FP32 pairs the running-average updates of consecutive accepted attempts (one pass for two,
    the older iterate read from the other buffer, a pending one applied before each evaluation);
    the same operations in the same order must give the same bits as one update per attempt: to
    tolerance (averages returned on some), at an iteration limit inside an evaluation interval
    (an update left pending), and for a batch."""
    cases = [(g.general_sparse(7, m=3000, n=6000, cap=1000), 1e-4, 400_000),
             (g.energy(4, T=96, N=8, K=6, E=16), 1e-4, 400_000),
             (g.multi_knapsack(1, m=150, n=400), 1e-6, 400_000),
             (g.energy(1, T=24, N=5, K=3, E=8), 0.0, 1037)]
    for lp, tol, lim in cases:
        got = []
        for single in (False, True):
            with pdlp.Problem(lp, precision="fp32", single_avg_updates=single) as p:
                info = p.solve(tol=tol, iter_limit=lim)
                got.append((p.get(), info))
        (a, ia), (b, ib) = got
        say("paired vs single updates:", lp.name, ia["iterations"], ib["iterations"], "average returned",
            ia["used_average"])
        assert (ia["iterations"], ia["restarts"], ia["used_average"]) == (ib["iterations"], ib["restarts"], ib["used_average"])
        assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y) and np.array_equal(a.rc, b.rc)
    lps = g.batch(3, count=16)
    out = []
    for single in (False, True):
        with pdlp.Batch(lps, precision="fp32", single_avg_updates=single) as bt:
            infos = bt.solve(tol=1e-4)
            out.append(([bt.get(i) for i in range(len(lps))], [f["iterations"] for f in infos]))
    assert out[0][1] == out[1][1]
    for sa, sb in zip(out[0][0], out[1][0]):
        assert np.array_equal(sa.x, sb.x) and np.array_equal(sa.y, sb.y)


def test_graphs_match_direct_launches(pdlp):
    lp = g.set_cover(2, m=800, n=2000)
    out = []
    for graphs in (True, False):
        with pdlp.Problem(lp, precision="fp32", use_graphs=graphs, tile_nnz=1024) as p:
            p.solve(tol=1e-4)
            out.append(p.get())
    assert np.array_equal(out[0].x, out[1].x) and out[0].info["iterations"] == out[1].info["iterations"]


def test_iteration_limit_and_warm_start(pdlp):
    lp = g.general_sparse(30, m=300, n=600, cap=100)
    f, xs, ys = P.highs(lp)
    with pdlp.Problem(lp, precision="fp64") as p:
        info = p.solve(tol=1e-8, iter_limit=50)
        assert info["status"] == pdlp.ITER_LIMIT and info["iterations"] == 50
        # warm start at the optimum: terminates at the first evaluation
        info = p.solve(tol=1e-7, x0=xs, y0=ys)
        assert info["status"] == pdlp.OPTIMAL and info["iterations"] == 64 and info["warm_started"] == 1
        # a garbage warm start is replaced by the cold start
        info = p.solve(tol=1e-4, x0=np.full(lp.n, 1e6), y0=np.full(lp.m, -1e6))
        assert info["fallback_used"] == 1 and info["status"] == pdlp.OPTIMAL


def test_fallback_keeps_or_resets_the_given_primal_weight(pdlp):
    """A rejected warm point is replaced by the cold point; with warm_fallback = 2 (default) the
    given omega0 stays, so the solve is bit for bit the cold solve started with that omega0, and with
    warm_fallback = 1 it is bit for bit the plain cold solve."""
    lp = g.set_cover(5, m=600, n=1500)
    bad_x, bad_y, om = np.full(lp.n, 1e6), np.full(lp.m, -1e6), 0.37
    for fb, ref_omega in ((2, om), (1, None)):
        with pdlp.Problem(lp, precision="fp32", warm_fallback=fb) as p:
            w = p.solve(tol=1e-4, x0=bad_x, y0=bad_y, omega0=om)
            sw = p.get()
            c = p.solve(tol=1e-4, omega0=ref_omega) if ref_omega else p.solve(tol=1e-4)
            sc = p.get()
        say("fallback", fb, w["iterations"], c["iterations"])
        assert w["fallback_used"] == 1 and w["status"] == pdlp.OPTIMAL
        assert w["iterations"] == c["iterations"]
        assert np.array_equal(sw.x, sc.x) and np.array_equal(sw.y, sc.y)


def test_device_memory_cap(pdlp):
    lp = g.set_cover(1, m=500, n=1000)
    with pytest.raises(pdlp.PDLPError) as e:
        pdlp.Problem(lp, device_mem_limit=4096)
    assert e.value.code == -3


def test_batch_matches_single(pdlp):
    """Each instance's chunks and work blocks depend on it alone: bitwise the single solve. The
    general sparse member is large enough for dozens of work blocks per side."""
    lps = [g.set_cover(10, m=300, n=700), g.general_sparse(11, m=200, n=500, cap=60),
           g.multi_knapsack(12, m=150, n=400), g.general_sparse(13, m=6000, n=12000, cap=800)]
    singles = []
    for lp in lps:
        with pdlp.Problem(lp, precision="fp32", tile_nnz=1024) as p:
            p.solve(tol=1e-4)
            singles.append(p.get())
    with pdlp.Batch(lps, precision="fp32", tile_nnz=1024) as bt:
        bt.solve(tol=1e-4)
        for i, lp in enumerate(lps):
            s = bt.get(i)
            say("batch", i, s.info["iterations"], singles[i].info["iterations"])
            assert s.info["iterations"] == singles[i].info["iterations"]
            assert np.array_equal(s.x, singles[i].x) and np.array_equal(s.y, singles[i].y)


def test_column_panel_product_parity(pdlp):
    """FP32 handles sum the long rows of A by column panels of x held in LDS (per-panel FP64 sums
    added in panel order). The product as the iteration forms it, against the oracle's: several
    panels with a ragged last one (n = 40,000 = 2 x 16,384 + 7,232), rows from 1 to 5,000 nonzeros
    (long rows in many row blocks, short ones through the chunks), the single-panel case, and a
    matrix whose long rows carry too few nonzeros to use panels; every row within one FP32 rounding
    of its FP64 sum (2e-6 of (|A||x|)_i)."""
    cases = [g.general_sparse(1, m=20000, n=40000), g.general_sparse(5, m=3000, n=9000, cap=2000),
             g.set_cover(2, m=800, n=2000)]
    rng = np.random.default_rng(3)
    for lp in cases:
        x = rng.standard_normal(lp.n)
        ref = oracle.spmv(lp.row_ptr, lp.col, lp.val, x)
        bound = 2e-6 * _absprod(lp, x) + 1e-30
        with pdlp.Problem(lp, precision="fp32", kernel_timing=True) as p:
            it = p.spmv(x, iteration=True)
            plain = p.spmv(x)
            p.solve(tol=0.0, iter_limit=64)
            launches = p.kernel_stats()["panel"]["launches"]
        with pdlp.Problem(lp, precision="fp32", panel_rows=-1, kernel_timing=True) as p:
            off = p.spmv(x, iteration=True)
            p.solve(tol=0.0, iter_limit=64)
            assert p.kernel_stats()["panel"]["launches"] == 0
        L = np.diff(lp.row_ptr)
        long_share = L[L >= 64].sum() / max(lp.nnz, 1)
        say("panels", lp.name, "long-row share %.2f" % long_share, "panel launches", launches,
            "max err / bound %.2e" % np.max(np.abs(it - ref) / bound))
        assert (launches > 0) == (long_share >= 0.5)
        assert np.all(np.abs(it - ref) <= bound)
        assert np.all(np.abs(plain - ref) <= bound) and np.all(np.abs(off - ref) <= bound)
    # a panel-sized x: exactly one panel, every column used
    m, n = 400, 16384
    rows, cols, vals = [], [], []
    for i in range(m):
        cs = rng.choice(n, size=int(rng.integers(64, 700)), replace=False)
        rows += [i] * cs.size
        cols += cs.tolist()
        vals += rng.standard_normal(cs.size).tolist()
    rp, ci, v = g._csr_from_triplets(m, n, rows, cols, vals)
    lp = g.LP(m, n, rp, ci, v, np.zeros(n), np.zeros(m), np.full(m, ord("E"), np.uint8),
              np.full(n, -np.inf), np.full(n, np.inf))
    x = rng.standard_normal(n)
    with pdlp.Problem(lp, precision="fp32") as p:
        it = p.spmv(x, iteration=True)
    ref = lp.to_scipy() @ x
    assert np.all(np.abs(it - ref) <= 2e-6 * _absprod(lp, x) + 1e-30)


def test_column_panels_in_a_batch_match_single_solves(pdlp):
    """Panels are built per instance: members with and without long rows solved in one batch give
    the bits of their single solves."""
    lps = [g.general_sparse(21, m=4000, n=20000, cap=3000), g.set_cover(22, m=500, n=1200),
           g.general_sparse(23, m=2500, n=40000, cap=4000)]
    singles = []
    for lp in lps:
        with pdlp.Problem(lp, precision="fp32", tile_nnz=1024) as p:
            p.solve(tol=1e-4, iter_limit=50_000)
            singles.append(p.get())
    with pdlp.Batch(lps, precision="fp32", tile_nnz=1024) as bt:
        bt.solve(tol=1e-4, iter_limit=50_000)
        for i in range(len(lps)):
            s = bt.get(i)
            say("panel batch", i, s.info["iterations"], singles[i].info["iterations"])
            assert s.info["iterations"] == singles[i].info["iterations"]
            assert np.array_equal(s.x, singles[i].x) and np.array_equal(s.y, singles[i].y)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_hard_general_seeds_reach_tolerance(pdlp, prec):
    """Seeds 8-10 of the 3,000 x 6,000 general family need 1e5 to 5e5 attempts in every
    implementation of the method: the FP64 oracle itself takes 77,312 / 326,400 / 116,544
    (tests/golden/general3k_oracle.json). Both precisions must reach 1e-4 as the oracle re-evaluates
    it within 2M attempts, with the objective in the weak-duality interval around HiGHS's optimum.
    The count itself is printed, not compared: rounding differences move the attempt at which the
    relative KKT error, hovering near 1e-4 for 1e4-1e5 attempts, first dips below it."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "general3k_oracle.json")))
    for seed in (8, 9, 10):
        lp = g.general_sparse(seed, m=3000, n=6000, cap=1000)
        ref = gold["seeds"][str(seed)]
        with pdlp.Problem(lp, precision=prec) as p:
            info = p.solve(tol=1e-4, iter_limit=2_000_000)
            sol = p.get()
        f, xs, ys = P.highs(lp)
        say("hard seed", seed, prec, info["status_name"], info["iterations"], "oracle", ref["iterations"],
            "obj rel to oracle %.2e" % (abs(info["primal_obj"] - ref["pobj"]) / abs(ref["pobj"])))
        assert info["status"] == pdlp.OPTIMAL and ref["status"] == oracle.OPTIMAL
        assert _objective_interval_ok(lp, sol.x, sol.y, f, xs, ys, f"seed {seed}")["rel_kkt"] <= 1e-4


def test_column_block_product_parity(pdlp):
    """FP32 handles may form A'y by column blocks: a work group owns 4,096 columns and reads y in
    16,384-row panels held in LDS, each column's run of entries in a panel summed in row order in
    FP64 and the panel sums added in panel order. The product as the iteration forms it, against the
    oracle's, with the path forced on: three row panels with a ragged last one and three column
    blocks with a ragged last one, columns of ~200 entries (runs longer than the two slots a group
    keeps in registers), short columns over 49 blocks (some columns empty), and the single-panel,
    single-block case; every entry within one FP32 rounding of its FP64 sum (2e-6 of (|A|'|y|)_j)."""
    cases = [g.general_sparse(31, m=40000, n=9000, cap=2000), g.general_sparse(32, m=40000, n=200000, cap=500),
             g.set_cover(2, m=800, n=2000)]
    rng = np.random.default_rng(4)
    for lp in cases:
        y = rng.standard_normal(lp.m)
        trp, tci, tv = oracle.transpose(lp.m, lp.n, lp.row_ptr, lp.col, lp.val)
        ref = oracle.spmv(trp, tci, tv, y)
        bound = 2e-6 * oracle.spmv(trp, tci, np.abs(tv), np.abs(y)) + 1e-30
        with pdlp.Problem(lp, precision="fp32", col_blocks=1, kernel_timing=True) as p:
            it = p.spmv(y, trans=True, iteration=True)
            plain = p.spmv(y, trans=True)
            p.solve(tol=0.0, iter_limit=64)
            launches = p.kernel_stats()["col_blocks"]["launches"]
        with pdlp.Problem(lp, precision="fp32", col_blocks=-1, kernel_timing=True) as p:
            off = p.spmv(y, trans=True, iteration=True)
            p.solve(tol=0.0, iter_limit=64)
            assert p.kernel_stats()["col_blocks"]["launches"] == 0
        empty = int(np.sum(np.diff(trp) == 0))
        say("col blocks", lp.name, "empty columns", empty, "launches", launches,
            "max err / bound %.2e" % np.max(np.abs(it - ref) / bound))
        assert launches > 0
        assert np.all(np.abs(it - ref) <= bound)
        assert np.all(np.abs(plain - ref) <= bound) and np.all(np.abs(off - ref) <= bound)


def test_row_block_product_parity(pdlp):
    """An instance on column blocks with no column-panel rows and at most 8 column panels also forms
    A x by row blocks: a work group owns 4,096 rows and reads x in 16,384-column panels held in LDS,
    each row's run in a panel summed in column order in FP64, the panel sums added in panel order and
    the entries past the dense panels gathered. The product as the iteration forms it, against the
    oracle's: three row blocks and three column panels with ragged ends and rows up to 300 entries
    (runs past the eight-slot batches), exactly eight panels, the single-block single-panel case, and
    nine panels (the row-block path off, the chunk engine's product); every entry within one FP32
    rounding of its FP64 sum (2e-6 of (|A||x|)_i)."""
    cases = [(g.general_sparse(41, m=9000, n=40000, cap=300), True),
             (g.set_cover(42, m=5000, n=8 * 16384, k=4), True),
             (g.set_cover(2, m=800, n=2000), True),
             (g.set_cover(43, m=3000, n=8 * 16384 + 1, k=4), False)]
    rng = np.random.default_rng(5)
    for lp, on in cases:
        x = rng.standard_normal(lp.n)
        ref = oracle.spmv(lp.row_ptr, lp.col, lp.val, x)
        bound = 2e-6 * oracle.spmv(lp.row_ptr, lp.col, np.abs(lp.val), np.abs(x)) + 1e-30
        with pdlp.Problem(lp, precision="fp32", col_blocks=1, panel_rows=-1, kernel_timing=True) as p:
            it = p.spmv(x, iteration=True)
            plain = p.spmv(x)
            p.solve(tol=0.0, iter_limit=64)
            st = p.kernel_stats()
        say("row blocks", lp.name, "launches", st["row_blocks"]["launches"], "dual launches",
            st["dual"]["launches"], "max err / bound %.2e" % np.max(np.abs(it - ref) / bound))
        assert (st["row_blocks"]["launches"] > 0) == on
        assert st["row_blocks"]["launches"] in (0, st["dual"]["launches"])
        assert np.all(np.abs(it - ref) <= bound) and np.all(np.abs(plain - ref) <= bound)


def test_row_block_solves_reach_tolerance(pdlp):
    """Solves with A x by row blocks reach relative KKT 1e-4 as the oracle re-evaluates it, with
    the objective inside the weak-duality interval on the set covers (HiGHS takes minutes on the
    knapsack relaxation, so it has the KKT check alone); in a batch the row-block members keep the
    bits of their single solves."""
    lps = [g.batch_member(0, 6, m_lo=2000, m_hi=6000), g.set_cover(44, m=6000, n=15000, k=6),
           g.multi_knapsack(45, m=5000, n=12500)]
    singles = []
    for i, q in enumerate(lps):
        with pdlp.Problem(q, precision="fp32", col_blocks=1, kernel_timing=True) as p:
            info = p.solve(tol=1e-4, iter_limit=200_000)
            sol = p.get()
            rb = p.kernel_stats()["row_blocks"]["launches"]
        say("row blocks", q.name, info["status_name"], info["iterations"], "row-block launches", rb)
        assert rb > 0 and info["status"] == pdlp.OPTIMAL
        if i < 2:
            f, xs, ys = P.highs(q)
            assert _objective_interval_ok(q, sol.x, sol.y, f, xs, ys, "row blocks")["rel_kkt"] <= 1e-4
        else:
            assert oracle.kkt(q, sol.x, sol.y)["rel_kkt"] <= 1e-4
        singles.append(sol)
    with pdlp.Batch(lps, precision="fp32", col_blocks=1) as bt:
        bt.solve(tol=1e-4, iter_limit=200_000)
        for i in range(len(lps)):
            s = bt.get(i)
            assert s.info["iterations"] == singles[i].info["iterations"]
            assert np.array_equal(s.x, singles[i].x) and np.array_equal(s.y, singles[i].y)


def test_column_block_solves_reach_tolerance(pdlp):
    """Solves with A'y by column blocks (forced on) reach relative KKT 1e-4 as the oracle
    re-evaluates it, with the objective inside the weak-duality interval; a batch of members with and
    without column blocks gives each member the bits of its single solve (the layout, and with it
    every summation order, depends on the instance alone)."""
    lp = g.general_sparse(7, m=3000, n=6000, cap=1000)
    f, xs, ys = P.highs(lp)
    with pdlp.Problem(lp, precision="fp32", col_blocks=1) as p:
        info = p.solve(tol=1e-4, iter_limit=2_000_000)
        sol = p.get()
    say("col blocks general", info["status_name"], info["iterations"], info["primal_obj"], "highs", f)
    assert info["status"] == pdlp.OPTIMAL
    assert _objective_interval_ok(lp, sol.x, sol.y, f, xs, ys, "col blocks")["rel_kkt"] <= 1e-4
    lps = [g.general_sparse(33, m=20000, n=30000, cap=800), g.set_cover(34, m=500, n=1200),
           g.general_sparse(35, m=2500, n=9000, cap=400)]
    singles = []
    for q in lps:
        with pdlp.Problem(q, precision="fp32", tile_nnz=1024, col_blocks=1) as p:
            p.solve(tol=1e-4, iter_limit=50_000)
            singles.append(p.get())
    with pdlp.Batch(lps, precision="fp32", tile_nnz=1024, col_blocks=1) as bt:
        bt.solve(tol=1e-4, iter_limit=50_000)
        for i in range(len(lps)):
            s = bt.get(i)
            say("col block batch", i, s.info["iterations"], singles[i].info["iterations"])
            assert s.info["iterations"] == singles[i].info["iterations"]
            assert np.array_equal(s.x, singles[i].x) and np.array_equal(s.y, singles[i].y)
